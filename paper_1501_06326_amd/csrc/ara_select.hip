// ara_select.hip -- PML and TVaR from a Year Loss Table (section 2.3).
//
// PML(RP) is the k-th largest trial loss, k = max(1, floor(N / RP)); it is
// found by a most-significant-digit radix select over the bit patterns of the
// losses (non-negative IEEE floats order like their unsigned bit patterns;
// -0.0 is folded onto +0.0): 8-bit digits, one histogram pass and one select
// step per digit.  TVaR(RP) is the mean of the k largest losses: the sum of
// the losses strictly above the PML plus (k - their count) copies of the
// PML, accumulated in FP64 with a fixed reduction order (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara_kernels.h"

namespace ara {

struct SelState {
    uint64_t prefix, mask;
    int64_t krem, k;
};

constexpr int kSumBlocks = 512;

template <typename T>
struct KeyOf;
template <>
struct KeyOf<float> {
    using K = uint32_t;
    static constexpr int bits = 32;
    __device__ static K key(float v) {
        const uint32_t b = __float_as_uint(v);
        return b == 0x80000000u ? 0u : b;
    }
    __device__ static double value(uint64_t k) { return (double)__uint_as_float((uint32_t)k); }
};
template <>
struct KeyOf<double> {
    using K = uint64_t;
    static constexpr int bits = 64;
    __device__ static K key(double v) {
        const uint64_t b = (uint64_t)__double_as_longlong(v);
        return b == 0x8000000000000000ull ? 0ull : b;
    }
    __device__ static double value(uint64_t k) { return __longlong_as_double((long long)k); }
};

template <typename T>
__global__ __launch_bounds__(256) void k_hist(const T *__restrict__ y, int64_t n,
                                              const SelState *__restrict__ st, int shift,
                                              uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = (uint64_t)KeyOf<T>::key(y[i]);
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// One thread: pick the digit holding the k-th largest, clear the histogram.
__global__ void k_select_digit(SelState *st, int shift, uint32_t *hist) {
    int64_t krem = st->krem, cum = 0;
    int pick = 0;
    for (int b = 255; b >= 0; --b) {
        const int64_t c = hist[b];
        if (cum + c >= krem) { pick = b; break; }
        cum += c;
    }
    st->krem = krem - cum;
    st->prefix |= (uint64_t)pick << shift;
    st->mask |= (uint64_t)255 << shift;
    for (int b = 0; b < 256; ++b) hist[b] = 0;
}

__global__ void k_init_state(SelState *st, int64_t k, uint32_t *hist) {
    st->prefix = 0;
    st->mask = 0;
    st->krem = k;
    st->k = k;
    for (int b = 0; b < 256; ++b) hist[b] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_tail_sum(const T *__restrict__ y, int64_t n,
                                                  const SelState *__restrict__ st,
                                                  double *__restrict__ psum,
                                                  unsigned long long *__restrict__ pcnt) {
    __shared__ double s[256];
    __shared__ unsigned long long c[256];
    const uint64_t thr = st->prefix;
    double acc = 0.0;
    unsigned long long cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T v = y[i];
        if ((uint64_t)KeyOf<T>::key(v) > thr) {
            acc += (double)v;
            ++cnt;
        }
    }
    s[threadIdx.x] = acc;
    c[threadIdx.x] = cnt;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s[threadIdx.x] += s[threadIdx.x + d];
            c[threadIdx.x] += c[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        psum[blockIdx.x] = s[0];
        pcnt[blockIdx.x] = c[0];
    }
}

template <typename T>
__global__ void k_finish(const SelState *st, const double *psum, const unsigned long long *pcnt,
                         int nb, double *out, int r, int n_rp) {
    double s = 0.0;
    unsigned long long c = 0;
    for (int b = 0; b < nb; ++b) {
        s += psum[b];
        c += pcnt[b];
    }
    const double pml = KeyOf<T>::value(st->prefix);
    const int64_t k = st->k;
    out[r] = pml;
    out[n_rp + r] = (s + (double)(k - (int64_t)c) * pml) / (double)k;
}

size_t pml_scratch_bytes(int64_t n) {
    (void)n;
    return 256 * sizeof(uint32_t) + 64 + kSumBlocks * (sizeof(double) + sizeof(unsigned long long)) +
           256;
}

template <typename T>
static hipError_t run_select(const T *y, int64_t n, const int64_t *ks, int32_t n_rp, void *scratch,
                             double *d_out, hipStream_t s) {
    char *p = (char *)scratch;
    uint32_t *hist = (uint32_t *)p;
    SelState *st = (SelState *)(p + 256 * sizeof(uint32_t));
    double *psum = (double *)(p + 256 * sizeof(uint32_t) + 64);
    unsigned long long *pcnt = (unsigned long long *)(psum + kSumBlocks);
    int64_t gb = (n + 255) / 256;
    const int g = (int)(gb < 1024 ? (gb < 1 ? 1 : gb) : 1024);
    const int gs = (int)(gb < kSumBlocks ? (gb < 1 ? 1 : gb) : kSumBlocks);
    for (int r = 0; r < n_rp; ++r) {
        hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, ks[r], hist);
        for (int shift = KeyOf<T>::bits - 8; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(k_hist<T>, dim3(g), dim3(256), 0, s, y, n, st, shift, hist);
            hipLaunchKernelGGL(k_select_digit, dim3(1), dim3(1), 0, s, st, shift, hist);
        }
        hipLaunchKernelGGL(k_tail_sum<T>, dim3(gs), dim3(256), 0, s, y, n, st, psum, pcnt);
        hipLaunchKernelGGL(k_finish<T>, dim3(1), dim3(1), 0, s, st, psum, pcnt, gs, d_out, r, n_rp);
    }
    return hipGetLastError();
}

hipError_t launch_pml_tvar(const void *ylt, int32_t dtype, int64_t n, const int64_t *ks, int32_t n_rp,
                           void *scratch, double *d_out, hipStream_t s) {
    if (dtype == ARA_F64) return run_select<double>((const double *)ylt, n, ks, n_rp, scratch, d_out, s);
    return run_select<float>((const float *)ylt, n, ks, n_rp, scratch, d_out, s);
}

}  // namespace ara
