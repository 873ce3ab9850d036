// ara_select.hip -- PML and TVaR from a Year Loss Table (section 2.3).
//
// PML(RP) is the k-th largest trial loss, k = max(1, floor(N / RP)); it is
// found by a most-significant-digit radix select over the bit patterns of the
// losses (non-negative IEEE floats order like their unsigned bit patterns;
// -0.0 is folded onto +0.0): 8-bit digits, one histogram pass and one select
// step per digit.  TVaR(RP) is the mean of the k largest losses: the sum of
// the losses strictly above the PML plus (k - their count) copies of the
// PML, accumulated in FP64 with a fixed reduction order (deterministic).
//
// The exceedance-probability curve (the return-period losses of the report
// the paper names) is the whole YLT in descending order: a stable
// least-significant-digit radix sort over the inverted key patterns (8-bit
// digits; per pass a block histogram, one scan of the digit-major counts, and
// a scatter that ranks equal digits by wavefront ballots), followed by FP64
// running means of the sorted losses (the TVaR at every point).
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

// Return periods are selected together, up to kSelGroup per pass over the
// YLT: every digit pass histograms all of them in one launch (periods whose
// selections still share their prefix share one histogram) and one small
// launch picks their digits, so a group costs the same launches whatever its
// size.  Launch boundaries order the passes (a last-block-done handshake
// would need a device-wide fence in every block, which costs more here).
constexpr int kSelGroup = 8;

struct SelGroup {
    int64_t k[kSelGroup];
};

// Scratch layout of one group.
struct SelScratch {
    uint32_t *hist;                 // [kSelGroup][256]
    SelState *st;                   // [kSelGroup]
    double *psum;                   // [kSelGroup][kSumBlocks]
    unsigned long long *pcnt;       // [kSelGroup][kSumBlocks]
};

__global__ __launch_bounds__(256) void k_init_state(SelScratch sc, SelGroup g, int m) {
    for (int i = threadIdx.x; i < kSelGroup * 256; i += blockDim.x) sc.hist[i] = 0;
    if ((int)threadIdx.x < m) {
        SelState &s = sc.st[threadIdx.x];
        s.prefix = 0;
        s.mask = 0;
        s.krem = g.k[threadIdx.x];
        s.k = g.k[threadIdx.x];
    }
}

// One digit of the selection for the m periods of a group.
template <typename T>
__global__ __launch_bounds__(256) void k_hist(const T *__restrict__ y, int64_t n, SelScratch sc,
                                              int m, int shift) {
    __shared__ uint32_t h[kSelGroup][256];
    __shared__ uint64_t pre[kSelGroup], msk[kSelGroup];
    __shared__ int rep[kSelGroup];
    for (int i = threadIdx.x; i < kSelGroup * 256; i += blockDim.x) (&h[0][0])[i] = 0;
    if (threadIdx.x == 0) {
        for (int r = 0; r < m; ++r) {
            pre[r] = sc.st[r].prefix;
            msk[r] = sc.st[r].mask;
            rep[r] = r;
            for (int q = 0; q < r; ++q)
                if (rep[q] == q && pre[q] == pre[r] && msk[q] == msk[r]) { rep[r] = q; break; }
        }
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = (uint64_t)KeyOf<T>::key(y[i]);
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        for (int r = 0; r < m; ++r)
            if (rep[r] == r && (k & msk[r]) == pre[r]) atomicAdd(&h[r][d], 1u);
    }
    __syncthreads();
    for (int r = 0; r < m; ++r) {
        const uint32_t c = h[rep[r]][threadIdx.x];
        if (c) atomicAdd(&sc.hist[r * 256 + threadIdx.x], c);
    }
}

// One block of 256 threads: for each period, the digit holding its k-th
// largest, from the suffix sums of its histogram (bin b counts the keys with
// digit b; the k-th largest is in the bin where the suffix sum reaches krem);
// then the histograms are cleared for the next digit.
__global__ __launch_bounds__(256) void k_pick(SelScratch sc, int m, int shift) {
    __shared__ uint64_t sfx[257];
    for (int r = 0; r < m; ++r) {
        const int64_t krem = sc.st[r].krem;
        sfx[threadIdx.x] = sc.hist[r * 256 + threadIdx.x];
        if (threadIdx.x == 0) sfx[256] = 0;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const uint64_t t = threadIdx.x + d < 256 ? sfx[threadIdx.x + d] : 0;
            __syncthreads();
            sfx[threadIdx.x] += t;
            __syncthreads();
        }
        const int64_t here = (int64_t)sfx[threadIdx.x], above = (int64_t)sfx[threadIdx.x + 1];
        __syncthreads();
        if (here >= krem && above < krem) {
            SelState &st = sc.st[r];
            st.krem = krem - above;
            st.prefix |= (uint64_t)threadIdx.x << shift;
            st.mask |= (uint64_t)255 << shift;
        }
    }
    for (int i = threadIdx.x; i < kSelGroup * 256; i += blockDim.x) sc.hist[i] = 0;
}

// TVaR of the group: per block and period, the FP64 sum and the count of the
// losses strictly above the period's PML (a fixed tree per block).
template <typename T>
__global__ __launch_bounds__(256) void k_tail_sum(const T *__restrict__ y, int64_t n, SelScratch sc,
                                                  int m) {
    __shared__ double s[256];
    __shared__ unsigned long long c[256];
    __shared__ uint64_t thr[kSelGroup];
    if ((int)threadIdx.x < m) thr[threadIdx.x] = sc.st[threadIdx.x].prefix;
    __syncthreads();
    double acc[kSelGroup];
    unsigned long long cnt[kSelGroup];
#pragma unroll
    for (int r = 0; r < kSelGroup; ++r) {
        acc[r] = 0.0;
        cnt[r] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T v = y[i];
        const uint64_t k = (uint64_t)KeyOf<T>::key(v);
#pragma unroll
        for (int r = 0; r < kSelGroup; ++r) {
            if (r < m && k > thr[r]) {
                acc[r] += (double)v;
                ++cnt[r];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kSelGroup; ++r) {
        if (r >= m) break;
        s[threadIdx.x] = acc[r];
        c[threadIdx.x] = cnt[r];
        __syncthreads();
        for (int d = 128; d >= 1; d >>= 1) {
            if ((int)threadIdx.x < d) {
                s[threadIdx.x] += s[threadIdx.x + d];
                c[threadIdx.x] += c[threadIdx.x + d];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            sc.psum[r * kSumBlocks + blockIdx.x] = s[0];
            sc.pcnt[r * kSumBlocks + blockIdx.x] = c[0];
        }
        __syncthreads();
    }
}

// One block: the nb blocks' partials of each period staged in LDS, added in
// block order by one thread (the same order for every run), PML and TVaR out.
template <typename T>
__global__ __launch_bounds__(256) void k_tail_finish(SelScratch sc, int m, int nb,
                                                     double *__restrict__ out, int r0, int n_rp) {
    __shared__ double ps[kSumBlocks];
    __shared__ unsigned long long pc[kSumBlocks];
    for (int r = 0; r < m; ++r) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            ps[b] = sc.psum[r * kSumBlocks + b];
            pc[b] = sc.pcnt[r * kSumBlocks + b];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            unsigned long long q = 0;
            for (int b = 0; b < nb; ++b) {
                t += ps[b];
                q += pc[b];
            }
            const double pml = KeyOf<T>::value(sc.st[r].prefix);
            const int64_t k = sc.st[r].k;
            out[r0 + r] = pml;
            out[n_rp + r0 + r] = (t + (double)(k - (int64_t)q) * pml) / (double)k;
        }
        __syncthreads();
    }
}

size_t pml_scratch_bytes(int64_t n) {
    (void)n;
    return kSelGroup * 256 * sizeof(uint32_t) + kSelGroup * sizeof(SelState) +
           kSelGroup * kSumBlocks * (sizeof(double) + sizeof(unsigned long long));
}

template <typename T>
static hipError_t run_select(const T *y, int64_t n, const int64_t *ks, int32_t n_rp, void *scratch,
                             double *d_out, hipStream_t s) {
    char *p = (char *)scratch;
    SelScratch sc;
    sc.hist = (uint32_t *)p;
    p += kSelGroup * 256 * sizeof(uint32_t);
    sc.st = (SelState *)p;
    p += kSelGroup * sizeof(SelState);
    sc.psum = (double *)p;
    p += kSelGroup * kSumBlocks * sizeof(double);
    sc.pcnt = (unsigned long long *)p;
    int64_t gb = (n + 255) / 256;
    const int g = (int)(gb < 1024 ? (gb < 1 ? 1 : gb) : 1024);
    const int gs = (int)(gb < kSumBlocks ? (gb < 1 ? 1 : gb) : kSumBlocks);
    for (int r0 = 0; r0 < n_rp; r0 += kSelGroup) {
        const int m = n_rp - r0 < kSelGroup ? n_rp - r0 : kSelGroup;
        SelGroup grp;
        for (int r = 0; r < kSelGroup; ++r) grp.k[r] = r < m ? ks[r0 + r] : 1;
        hipLaunchKernelGGL(k_init_state, dim3(1), dim3(256), 0, s, sc, grp, m);
        for (int shift = KeyOf<T>::bits - 8; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(k_hist<T>, dim3(g), dim3(256), 0, s, y, n, sc, m, shift);
            hipLaunchKernelGGL(k_pick, dim3(1), dim3(256), 0, s, sc, m, shift);
        }
        hipLaunchKernelGGL(k_tail_sum<T>, dim3(gs), dim3(256), 0, s, y, n, sc, m);
        hipLaunchKernelGGL(k_tail_finish<T>, dim3(1), dim3(256), 0, s, sc, m, gs, d_out, r0, n_rp);
    }
    return hipGetLastError();
}

// ---- exceedance-probability curve ------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortIpt = 16;
constexpr int kSortTile = kSortThreads * kSortIpt;   // keys per block and pass

template <typename T>
__global__ void k_sort_keys(const T *__restrict__ y, int64_t n, typename KeyOf<T>::K *__restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        keys[i] = ~KeyOf<T>::key(y[i]);          // ascending inverted = descending losses
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const K *__restrict__ keys, int64_t n,
                                                            int shift, uint32_t *__restrict__ counts,
                                                            int nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortIpt; ++r) {
        const int64_t i = t0 + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit: the block's keys in kSortIpt rounds of 256 (in
// index order); in a round each wavefront finds the lanes sharing a lane's
// digit with eight ballots, the lowest of them records the count, and a key
// lands at its digit's block offset + the keys of that digit in earlier
// rounds and earlier wavefronts + its rank among its wavefront's equals.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const K *__restrict__ in,
                                                               K *__restrict__ out, int64_t n,
                                                               int shift,
                                                               const uint32_t *__restrict__ offs,
                                                               int nb) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    base[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    for (int q = 0; q < kSortThreads / 64; ++q) wcnt[q][tid] = 0u;
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortIpt; ++r) {
        const int64_t i = t0 + (int64_t)r * kSortThreads + tid;
        const bool valid = i < n;
        const K k = valid ? in[i] : (K)0;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t b = __ballot(valid && on);
            m &= on ? b : ~b;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0u) wcnt[w][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            out[pos] = k;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int q = 0; q < kSortThreads / 64; ++q) {
            add += wcnt[q][tid];
            wcnt[q][tid] = 0u;
        }
        base[tid] += add;
        __syncthreads();
    }
}

template <typename T>
__global__ void k_sort_values(typename KeyOf<T>::K *__restrict__ keys, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = KeyOf<T>::value(~keys[i]);
        reinterpret_cast<T *>(keys)[i] = (T)v;
    }
}

// Running means of the sorted losses in FP64: block sums, a scan of them, and
// a block-local scan (a serial run of kSortIpt per thread).
template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_tm_partial(const T *__restrict__ v, int64_t n,
                                                             double *__restrict__ part) {
    __shared__ double s[kSortThreads];
    const int64_t b0 = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortIpt;
    double acc = 0.0;
    for (int j = 0; j < kSortIpt; ++j)
        if (b0 + j < n) acc += (double)v[b0 + j];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int d = kSortThreads / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Exclusive scan of the block sums in block order (one thread adds, so the
// order is fixed); tiles of them are staged through LDS by the whole block.
__global__ __launch_bounds__(kSortThreads) void k_tm_scan(double *__restrict__ part, int nb) {
    constexpr int kT = kSortThreads * 8;
    __shared__ double t[kT];
    __shared__ double carry;
    if (threadIdx.x == 0) carry = 0.0;
    for (int b0 = 0; b0 < nb; b0 += kT) {
        const int m = nb - b0 < kT ? nb - b0 : kT;
        for (int i = threadIdx.x; i < m; i += blockDim.x) t[i] = part[b0 + i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double run = carry;
            for (int i = 0; i < m; ++i) {
                const double v = t[i];
                t[i] = run;
                run += v;
            }
            carry = run;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) part[b0 + i] = t[i];
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_tm_final(const T *__restrict__ v, int64_t n,
                                                           const double *__restrict__ part,
                                                           double *__restrict__ tm) {
    __shared__ double s[kSortThreads];
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kSortTile + (int64_t)tid * kSortIpt;
    double acc = 0.0;
    for (int j = 0; j < kSortIpt; ++j)
        if (b0 + j < n) acc += (double)v[b0 + j];
    s[tid] = acc;
    __syncthreads();
    for (int d = 1; d < kSortThreads; d <<= 1) {
        const double x = tid >= d ? s[tid - d] : 0.0;
        __syncthreads();
        s[tid] += x;
        __syncthreads();
    }
    double run = part[blockIdx.x] + (tid ? s[tid - 1] : 0.0);
    for (int j = 0; j < kSortIpt; ++j) {
        const int64_t i = b0 + j;
        if (i < n) {
            run += (double)v[i];
            tm[i] = run / (double)(i + 1);
        }
    }
}

static int sort_blocks(int64_t n) { return (int)((n + kSortTile - 1) / kSortTile); }

size_t ep_scratch_bytes(int64_t n, int32_t dtype) {
    const size_t ks = dtype == ARA_F64 ? 8 : 4;
    const size_t nb = (size_t)sort_blocks(n > 0 ? n : 1);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return up(ks * (size_t)(n > 0 ? n : 1)) + up(sizeof(uint32_t) * 256 * nb) + up(sizeof(double) * nb);
}

template <typename T>
static hipError_t run_ep(const T *y, int64_t n, T *sorted, double *tail_mean, void *scratch,
                         hipStream_t s) {
    using K = typename KeyOf<T>::K;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int nb = sort_blocks(n);
    char *p = (char *)scratch;
    K *tmp = (K *)p;
    uint32_t *counts = (uint32_t *)(p + up(sizeof(K) * (size_t)n));
    double *part = (double *)((char *)counts + up(sizeof(uint32_t) * 256 * (size_t)nb));
    K *keys = (K *)sorted;                        // the output doubles as a key buffer
    const int g = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL((k_sort_keys<T>), dim3(g), dim3(256), 0, s, y, n, keys);
    K *a = keys, *b = tmp;
    for (int shift = 0; shift < KeyOf<T>::bits; shift += 8) {   // an even number of passes
        hipLaunchKernelGGL((k_sort_hist<K>), dim3(nb), dim3(kSortThreads), 0, s, a, n, shift,
                           counts, nb);
        launch_scan_excl_u32(counts, (int64_t)256 * nb, s);
        hipLaunchKernelGGL((k_sort_scatter<K>), dim3(nb), dim3(kSortThreads), 0, s, a, b, n,
                           shift, counts, nb);
        K *t = a;
        a = b;
        b = t;
    }
    hipLaunchKernelGGL((k_sort_values<T>), dim3(g), dim3(256), 0, s, keys, n);
    if (tail_mean) {
        hipLaunchKernelGGL((k_tm_partial<T>), dim3(nb), dim3(kSortThreads), 0, s, sorted, n, part);
        hipLaunchKernelGGL(k_tm_scan, dim3(1), dim3(kSortThreads), 0, s, part, nb);
        hipLaunchKernelGGL((k_tm_final<T>), dim3(nb), dim3(kSortThreads), 0, s, sorted, n, part,
                           tail_mean);
    }
    return hipGetLastError();
}

hipError_t launch_ep_curve(const void *ylt, int32_t dtype, int64_t n, void *sorted,
                           double *tail_mean, void *scratch, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dtype == ARA_F64)
        return run_ep<double>((const double *)ylt, n, (double *)sorted, tail_mean, scratch, s);
    return run_ep<float>((const float *)ylt, n, (float *)sorted, tail_mean, scratch, s);
}

hipError_t launch_pml_tvar(const void *ylt, int32_t dtype, int64_t n, const int64_t *ks, int32_t n_rp,
                           void *scratch, double *d_out, hipStream_t s) {
    if (dtype == ARA_F64) return run_select<double>((const double *)ylt, n, ks, n_rp, scratch, d_out, s);
    return run_select<float>((const float *)ylt, n, ks, n_rp, scratch, d_out, s);
}

}  // namespace ara
