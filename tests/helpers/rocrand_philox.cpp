// Host-side driver for rocRAND's Philox4x32-10 engine, used only by the tests
// as an implementation independent of both the oracle and the GPU library.
// It calls the installed rocRAND header's engine (ten_rounds on a raw
// counter/key); nothing of rocRAND is copied here.
#include <rocrand/rocrand_philox4x32_10.h>

namespace {
struct RawPhilox : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
}  // namespace

extern "C" void rr_philox_batch(long long n, const unsigned *ctr, const unsigned *key,
                                unsigned *out)
{
    RawPhilox eng;
    uint2 k;
    k.x = key[0];
    k.y = key[1];
    for (long long j = 0; j < n; ++j) {
        uint4 c;
        c.x = ctr[4 * j + 0]; c.y = ctr[4 * j + 1]; c.z = ctr[4 * j + 2]; c.w = ctr[4 * j + 3];
        uint4 r = eng.apply(c, k);
        out[4 * j + 0] = r.x; out[4 * j + 1] = r.y; out[4 * j + 2] = r.z; out[4 * j + 3] = r.w;
    }
}
