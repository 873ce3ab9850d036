// ara_kernels.hip -- gfx950 kernels of Aggregate Risk Analysis.
//
//  * YET validation (section 2.1 (i)).
//  * Portfolio build (sections 3.3 and 4.2): per-ELT direct-access tables over
//    the catalogue, the per-layer event-major row lists, the per-row Beta
//    moment fit, and (without secondary uncertainty) the per-event
//    occurrence-loss table.
//  * The analysis (Algorithm 1 with secondary uncertainty):
//      - k_ara_pu: primary uncertainty only.  The loss of an occurrence is
//        then a function of its event id alone, so the layer's per-event
//        occurrence losses are tabulated once (lookup, ELT terms, cross-ELT
//        sum and occurrence terms for every catalogue event) and a trial is a
//        gather-sum over its event ids followed by the aggregate terms.
//      - k_ara_su: secondary uncertainty.  One wavefront per trial; lanes
//        read consecutive occurrences, look each up in the layer's event-major
//        rows, and append the hits to an LDS queue (the fast pass only the
//        rows that can pay: the others add exactly 0); the queue is drained
//        64 hits at a time so every lane of a batch draws, inverts the Beta
//        CDF and applies the ELT terms on real work (the paper's
//        "convergence switching" idea applied to SIMD lanes).  A trial with
//        a hit that needs the FP64 quantile (tail band, shapes outside the
//        FP32 domain, the two-normal mix, FP32 non-convergence) is handed to
//        k_ara_su_redo, which runs it again with the FP64 path in place
//        (k_ara_su_redo4: the same code in a 4-wavefront register budget,
//        for portfolios with FP64-quantile rows and no mixed rows).
//      - k_ara_batch / k_ara_batch_items: the same trial code over
//        (portfolio, trial tile) work items of many portfolios at once.
//      - the occurrence view (per-occurrence increments of the aggregate
//        terms): the OCC instantiation of k_ara_su, or k_pu_occ_view without
//        secondary uncertainty, both through occ_chunk's wavefront scan.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara_internal.h"
#include "ara_math.h"
#include "ara_kernels.h"

namespace ara {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void report(Status *st, int32_t code, int64_t a, int64_t b, int64_t c) {
    if (atomicCAS(&st->code, 0, code) == 0) {
        st->where[0] = a;
        st->where[1] = b;
        st->where[2] = c;
    }
}

__device__ __forceinline__ float clampf_terms(float x, float r, float l) {
    return fminf(fmaxf(x - r, 0.0f), l);
}
__device__ __forceinline__ double clampd_terms(double x, double r, double l) {
    return fmin(fmax(x - r, 0.0), l);
}

// exclusive prefix sum of v over the 64 lanes of the wavefront (lane order)
__device__ __forceinline__ int wave_excl_scan(int v, int *total) {
    // Inclusive prefix sum over the wavefront with DPP moves: shifts within
    // each row of 16 lanes (lanes shifted in from outside the row read 0),
    // then lane 15 of rows 0 and 2 added into rows 1 and 3, then lane 31
    // added into rows 2 and 3 (the other rows keep the 0 given as old).
    int s = v;
    s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xf, 0xf, true);   // row_shr:1
    s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xf, 0xf, true);   // row_shr:2
    s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xf, true);   // row_shr:4
    s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xf, true);   // row_shr:8
    s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xa, 0xf, false);  // row_bcast:15
    s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xc, 0xf, false);  // row_bcast:31
    *total = __builtin_amdgcn_readlane(s, 63);
    return s - v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Sum accumulators for a trial's occurrence losses (ara_run_opts.sum_mode).
template <int MODE>
struct Acc;
template <>
struct Acc<ARA_SUM_NAIVE32> {
    float s = 0.0f;
    __device__ void add(float v) { s += v; }
    __device__ double total() {
        float t = s;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        return (double)t;
    }
};
template <>
struct Acc<ARA_SUM_KAHAN32> {
    float s = 0.0f, c = 0.0f;   // Neumaier: exact sum = s + c (up to c's rounding)
    __device__ void add(float v) {
        const float t = s + v;
        c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
        s = t;
    }
    __device__ double total() {
        float S = s, C = c;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const float So = __shfl_xor(S, d, 64), Co = __shfl_xor(C, d, 64);
            // both lanes of a pair compute the same combination (symmetric order)
            const float a = fmaxf(fabsf(S), fabsf(So)) == fabsf(S) ? S : So;
            const float b = (a == S) ? So : S;
            const float t = a + b;
            const float e = (a - t) + b;
            C = C + Co + e;
            S = t;
        }
        return (double)S + (double)C;
    }
};
template <>
struct Acc<ARA_SUM_F64> {
    double s = 0.0;
    __device__ void add(float v) { s += (double)v; }
    __device__ double total() {
        double t = s;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        return t;
    }
};

// ---------------------------------------------------------------------------
// YET validation: one wavefront per trial
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_validate_yet(const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ ev,
                                                      const float *__restrict__ times,
                                                      int64_t n_trials, int32_t n_cat,
                                                      Status *st, unsigned long long *max_len) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
    if (wid == 0 && lane == 0 && off[0] != 0) report(st, ARA_E_OFFSETS_NOT_MONOTONE, 0, off[0], 0);
    const int64_t n_occ = off[n_trials];
    unsigned long long longest = 0;   // this wavefront's longest trial (one atomic per wavefront)
    for (int64_t t = wid; t < n_trials; t += nw) {
        const int64_t a = off[t], b = off[t + 1];
        // a trial is read only when it lies inside [0, offsets[n_trials])
        if (a < 0 || b < a || b > n_occ) {
            if (lane == 0) report(st, ARA_E_OFFSETS_NOT_MONOTONE, t, a, b);
            continue;
        }
        if ((unsigned long long)(b - a) > longest) longest = (unsigned long long)(b - a);
        // four ids (and time pairs) in flight per lane: every load takes an
        // index inside the trial (a lane past its end reads its first
        // element) so they issue together; the checks use the real index
        for (int64_t j0 = a + lane; j0 < b; j0 += 4 * 64) {
            int32_t e[4];
            float t0[4], t1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = j0 + 64 * u;
                const int64_t jj = j < b ? j : a;
                e[u] = ev[jj];
                if (times) {
                    t0[u] = times[jj];
                    t1[u] = times[jj + 1 < b ? jj + 1 : jj];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = j0 + 64 * u;
                if (j < b && (e[u] < 0 || e[u] >= n_cat))
                    report(st, ARA_E_EVENT_ID_RANGE, t, j - a, e[u]);
                if (times && j + 1 < b && !(t0[u] <= t1[u]))
                    report(st, ARA_E_TIMES_UNSORTED, t, j - a, 0);
            }
        }
    }
    if (lane == 0 && longest > 0) atomicMax(max_len, longest);
}

// ---------------------------------------------------------------------------
// portfolio build
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Row checks that need no other row: finite, non-negative, mean < max_loss
// where the row has secondary uncertainty, event id in range.
__global__ void k_check_rows(const RawRow *__restrict__ raw, int64_t n, int32_t n_cat,
                             int32_t su, Status *st) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const RawRow r = raw[i];
        bool bad = !(r.mean >= 0.0f && r.sigma_i >= 0.0f && r.sigma_c >= 0.0f) ||
                   !isfinite(r.mean) || !isfinite(r.sigma_i) || !isfinite(r.sigma_c);
        if (su && (r.sigma_i + r.sigma_c) > 0.0f)
            bad = bad || !(r.max_loss > r.mean) || !isfinite(r.max_loss);
        if (r.event < 0 || r.event >= n_cat) report(st, ARA_E_EVENT_ID_RANGE, -1, i, r.event);
        else if (bad) report(st, ARA_E_BAD_ELT_ROW, -1, i, 0);
    }
}

// Direct-access tables of one layer: dat[j * n_cat + event] = raw row index
// for the layer's ELT j (section 4.2).  A second row for the same event in
// one ELT is a duplicate.
__global__ void k_dat_scatter(const RawRow *__restrict__ raw, const int64_t *__restrict__ elt_row_off,
                              int32_t elt_begin, int32_t n_elts, int32_t n_cat,
                              int32_t *__restrict__ dat, Status *st) {
    const int64_t r0 = elt_row_off[elt_begin], r1 = elt_row_off[elt_begin + n_elts];
    for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1;
         r += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_elts - 1;   // ELT of row r
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (elt_row_off[elt_begin + mid] <= r) lo = mid; else hi = mid - 1;
        }
        const int32_t e = raw[r].event;
        if (e < 0 || e >= n_cat) continue;
        const int32_t old = atomicCAS(&dat[(int64_t)lo * n_cat + e], -1, (int32_t)(r - r0));
        if (old != -1) report(st, ARA_E_BAD_ELT_ROW, -2, r, e);
    }
}

// A row whose ELT terms give 0 for every draw: a loss never exceeds its
// scale (max_l, or the mean when there is no draw), so scale <= retention,
// a zero limit or a zero share make share * min(max(loss - R, 0), L)
// exactly 0.
__device__ __forceinline__ bool row_cannot_pay(const RawRow &rr, const EltDev &ed, int32_t su) {
    const bool det = !su || (double)rr.sigma_i + (double)rr.sigma_c == 0.0;
    const float scale = det ? rr.mean : rr.max_loss;
    return scale <= ed.retention || ed.limit == 0.0f || ed.share == 0.0f;
}

// Rows per catalogue event in the layer (evoff) and rows that can pay (liveoff).
__global__ void k_ev_count(const int32_t *__restrict__ dat, const RawRow *__restrict__ raw,
                           const int64_t *__restrict__ elt_row_off, const EltDev *__restrict__ elts,
                           int32_t elt_begin, int32_t n_elts, int32_t n_cat, int32_t su,
                           uint32_t *__restrict__ evoff, uint32_t *__restrict__ liveoff) {
    for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e <= n_cat; e += gridDim.x * blockDim.x) {
        uint32_t c = 0, live = 0;
        if (e < n_cat)
            for (int j = 0; j < n_elts; ++j) {
                const int32_t r = dat[(int64_t)j * n_cat + e];
                if (r < 0) continue;
                ++c;
                live += row_cannot_pay(raw[elt_row_off[elt_begin] + r], elts[elt_begin + j], su)
                            ? 0u : 1u;
            }
        evoff[e] = c;
        liveoff[e] = live;
    }
}

// In-place exclusive scan of n values with one 1024-thread block: rounds of
// 8 tiles of 1024 values, loaded together (coalesced) and scanned tile by
// tile in order with a wavefront scan and the 16 wavefront totals in LDS.
__global__ __launch_bounds__(1024) void k_scan_excl_u32(uint32_t *p, int64_t n) {
    constexpr int kTiles = 8;
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t carry = 0;                          // sum of everything before the round
    for (int64_t base = 0; base < n; base += (int64_t)kTiles * 1024) {
        uint32_t v[kTiles];
#pragma unroll
        for (int k = 0; k < kTiles; ++k) {
            const int64_t i = base + (int64_t)k * 1024 + tid;
            v[k] = i < n ? p[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kTiles; ++k) {
            int wt;
            // the bits of a uint32 sum are those of the int32 sum
            const uint32_t ex = (uint32_t)wave_excl_scan((int)v[k], &wt);
            if (lane == 0) wsum[w] = (uint32_t)wt;
            __syncthreads();
            uint32_t before = 0, tile = 0;
            for (int q = 0; q < 16; ++q) {
                const uint32_t t = wsum[q];
                before += q < w ? t : 0u;
                tile += t;
            }
            const int64_t i = base + (int64_t)k * 1024 + tid;
            if (i < n) p[i] = carry + before + ex;
            carry += tile;
            __syncthreads();
        }
    }
}

// Beta moment fit of section 3.3 in FP64, then rounded shape parameters.
__device__ void fit_row(const RawRow &r, int32_t su, RowQ *q, uint32_t *flags, float *cfrac,
                        double *lnb64) {
    const double mu = r.mean, si = r.sigma_i, sc = r.sigma_c, mx = r.max_loss;
    const double sigma = si + sc;
    *cfrac = 0.0f;
    if (!su || sigma == 0.0) {
        *flags = ROW_DET;
        q->scale = r.mean;
        q->a = q->b = q->lnb = 0.0f;
        *lnb64 = 0.0;
        return;
    }
    const double mu_b = mu / mx;
    double s_b = sigma / mx;
    const double s_max = sqrt(mu_b * (1.0 - mu_b));
    bool capped = false;
    if (s_b >= s_max) {
        s_b = (1.0 - 1e-6) * s_max;
        capped = true;
    }
    const double rr = s_max / s_b;
    const double kappa = rr * rr - 1.0;
    const float a = (float)(mu_b * kappa), b = (float)((1.0 - mu_b) * kappa);
    const double lnb = lgamma((double)a) + lgamma((double)b) - lgamma((double)a + (double)b);
    q->scale = r.max_loss;
    q->a = a;
    q->b = b;
    q->lnb = (float)(lnb * 1.4426950408889634);   // log2 B(a, b)
    *lnb64 = lnb;
    uint32_t f = 0;
    if (capped || !(a >= kF32MinShape && b >= kF32MinShape && a <= kF32MaxShape &&
                    b <= kF32MaxShape)) {
        f |= ROW_F64;
    } else {
        const int na = cf_terms((double)a, (double)b), nb = cf_terms((double)b, (double)a);
        if (na == 0 || nb == 0) f |= ROW_F64;
        else f |= ((uint32_t)na << 20) | ((uint32_t)nb << 26);
    }
    if (si > 0.0 && sc > 0.0) {
        f |= ROW_CORR;
        *cfrac = (float)(sc / sigma);
    } else if (si == 0.0) {
        f |= ROW_CONLY;
    }
    *flags = f;
}

// The Beta fit of every raw row of the portfolio, one thread per row: the
// fit (FP64 moment fit, ln B and the continued-fraction term counts) is the
// costly part of the build and does not depend on where the row lands.
__global__ void k_fit_rows(const RawRow *__restrict__ raw, int64_t n, int32_t su,
                           RowFit *__restrict__ fit) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        RowFit f;
        fit_row(raw[i], su, &f.q, &f.flags, &f.cfrac, &f.lnb);
        fit[i] = f;
    }
}

// Event-major rows of one layer: for every catalogue event, its rows in the
// layer's ELT order, with the fitted Beta constants; also the per-event
// occurrence loss table when secondary uncertainty is off.
__global__ void k_ev_fill(const int32_t *__restrict__ dat, const RawRow *__restrict__ raw,
                          const RowFit *__restrict__ fit,
                          const int64_t *__restrict__ elt_row_off, const EltDev *__restrict__ elts,
                          LayerDev *__restrict__ layer, int32_t n_cat, int32_t su,
                          const uint32_t *__restrict__ evoff, uint32_t *__restrict__ live_out,
                          const uint32_t *__restrict__ liveoff, RowQ *__restrict__ rowq,
                          RowF *__restrict__ rowf,
                          float *__restrict__ row_mean, float *__restrict__ row_cfrac,
                          uint32_t *__restrict__ row_meta, double *__restrict__ row_lnb,
                          float *__restrict__ otab) {
    const LayerDev L = *layer;
    uint32_t fl_or = 0;
    for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_cat; e += gridDim.x * blockDim.x) {
        int64_t pos = L.row_base + evoff[e];
        int64_t fpos = L.row_base + liveoff[e];       // compact record of the next paying row
        uint32_t live = 0;
        float X = 0.0f;
        // rows that can pay first, then the rows whose ELT terms give 0 for
        // every draw (row_cannot_pay)
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < L.n_elts; ++j) {
                const int32_t r = dat[(int64_t)j * n_cat + e];
                if (r < 0) continue;
                const int64_t ri = elt_row_off[L.elt_begin] + r;
                const RawRow rr = raw[ri];
                const EltDev ed = elts[L.elt_begin + j];
                const bool dead = row_cannot_pay(rr, ed, su);
                if (dead != (pass == 1)) continue;
                const RowFit rf = fit[ri];
                const RowQ q = rf.q;
                const uint32_t f = rf.flags;
                const float cf = rf.cfrac;
                const double lb = rf.lnb;
                row_lnb[pos] = lb;
                rowq[pos] = q;
                row_mean[pos] = rr.mean;
                row_cfrac[pos] = cf;
                row_meta[pos] = f | (uint32_t)j;
                fl_or |= f & ROW_FLAGS;
                if (!dead) {
                    RowF F;
                    F.scale = q.scale;
                    F.meta = f | (uint32_t)j;
                    F.rs = (uint32_t)(pos - L.row_base) << 5;   // shape set by k_shape_assign
                    F.cfrac = cf;
                    rowf[fpos++] = F;
                }
                ++pos;
                live += dead ? 0u : 1u;
                X += ed.share * clampf_terms(rr.mean, ed.retention, ed.limit);
            }
        live_out[2 * e] = liveoff[e];
        live_out[2 * e + 1] = live;
        if (otab) otab[L.otab_base + e] = clampf_terms(X, L.occ_r, L.occ_l);
    }
    if (fl_or) atomicOr(&layer->flags, fl_or);
}

// ---------------------------------------------------------------------------
// primary uncertainty: per-event occurrence-loss table, gather-sum per trial
// ---------------------------------------------------------------------------
// Sparse form of a layer's otab: bit w*32+i of bits[] set when otab is
// non-zero, rank[w] = set bits before word w (exclusive scan), vals[] the
// non-zero values in event order.  Lookup of event E: one LDS word, and for
// the (rare) non-zero events the rank and the value.
__global__ void k_sp_bits(const float *__restrict__ otab, int32_t n_cat, uint32_t *__restrict__ bits,
                          uint32_t *__restrict__ rank) {
    const int32_t nw = (n_cat + 31) >> 5;
    for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w <= nw; w += gridDim.x * blockDim.x) {
        uint32_t b = 0;
        if (w < nw)
            for (int i = 0; i < 32; ++i) {
                const int32_t e = w * 32 + i;
                if (e < n_cat && otab[e] != 0.0f) b |= 1u << i;
            }
        if (w < nw) bits[w] = b;
        rank[w] = __popc(b);
    }
}

__global__ void k_sp_vals(const float *__restrict__ otab, int32_t n_cat,
                          const uint32_t *__restrict__ bits, const uint32_t *__restrict__ rank,
                          float *__restrict__ vals, LayerDev *layer) {
    const int32_t nw = (n_cat + 31) >> 5;
    for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
        uint32_t b = bits[w], r = rank[w];
        while (b) {
            const int i = __ffs(b) - 1;
            vals[r++] = otab[w * 32 + i];
            b &= b - 1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) layer->nnz = (int32_t)rank[nw];
}

struct PuArgs {
    const int64_t *off;
    const int32_t *ev;
    int64_t trial_begin, trial_count;
    const float *otab;
    const uint32_t *sp_bits, *sp_rank;
    const float *sp_vals;
    int32_t nnz, n_cat;
    float agg_r, agg_l;
    int32_t layer;
    void *ylt_layers, *ylt_pf;
    int32_t accumulate_pf;
    void *occ_view;
    int64_t occ_stride;
    Status *status;
};

enum { TAB_GLOBAL = 0, TAB_LDS_DENSE = 1, TAB_LDS_SPARSE = 2 };

// Occurrence view of 64 consecutive occurrences of one trial and layer, in
// stored order: o (lane's occurrence loss net of the occurrence terms, 0 past
// the end) is scanned into the running sum S (FP64, carried in *cs), the
// aggregate terms give A = min(max(S - AggR, 0), AggL) (carried in *ca), and
// the lane's increment A - A_prev is written at pos when valid.  Every lane
// of the wave calls this (the scan reads all of them).
// A DPP move of an FP64 value (both 32-bit halves with the same control);
// lanes that receive nothing read 0.0.
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xf, BOUND);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xf, BOUND);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <bool F64OUT>
__device__ __forceinline__ void occ_chunk(double o, bool valid, int64_t pos, int layer,
                                          void *view, int64_t stride, float agg_r, float agg_l,
                                          double *cs, double *ca, Status *st, int64_t trial) {
    const int lane = threadIdx.x & 63;
    // inclusive FP64 prefix sum over the wavefront, laid out as in wave_excl_scan
    o += dpp_f64<0x111, 0xf, true>(o);    // row_shr:1
    o += dpp_f64<0x112, 0xf, true>(o);    // row_shr:2
    o += dpp_f64<0x114, 0xf, true>(o);    // row_shr:4
    o += dpp_f64<0x118, 0xf, true>(o);    // row_shr:8
    o += dpp_f64<0x142, 0xa, false>(o);   // row_bcast:15
    o += dpp_f64<0x143, 0xc, false>(o);   // row_bcast:31
    const double S = *cs + o;
    const double A = clampd_terms(S, (double)agg_r, (double)agg_l);
    double Ap = __shfl_up(A, 1, 64);
    if (lane == 0) Ap = *ca;
    if (valid) {
        if (pos < stride) {
            const int64_t at = (int64_t)layer * stride + pos;
            if (F64OUT) ((double *)view)[at] = A - Ap;
            else ((float *)view)[at] = (float)(A - Ap);
        } else {
            report(st, ARA_E_WORKSPACE_TOO_SMALL, trial, pos, stride);
        }
    }
    *cs = readlane_f64(S, 63);
    *ca = readlane_f64(A, 63);
}

// The layer's per-event occurrence-loss table, staged by the whole block in
// LDS (dense, or sparse: a bit per event, the rank of each 32-event word and
// the non-zero values) or read from global memory (catalogues too large).
template <int TAB>
__device__ __forceinline__ void pu_stage_table(const PuArgs &P, uint32_t *sm) {
    const int32_t nw = (P.n_cat + 31) >> 5;
    if (TAB == TAB_LDS_DENSE) {
        float *tab = (float *)sm;
        for (int i = threadIdx.x; i < P.n_cat; i += blockDim.x) tab[i] = P.otab[i];
    } else if (TAB == TAB_LDS_SPARSE) {
        uint32_t *bits = sm, *rank = sm + nw;
        float *vals = (float *)(sm + 2 * nw + 1);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) bits[i] = P.sp_bits[i];
        for (int i = threadIdx.x; i <= nw; i += blockDim.x) rank[i] = P.sp_rank[i];
        for (int i = threadIdx.x; i < P.nnz; i += blockDim.x) vals[i] = P.sp_vals[i];
    }
    if (TAB != TAB_GLOBAL) __syncthreads();
}

template <int TAB>
__device__ __forceinline__ float pu_look(const PuArgs &P, const uint32_t *sm, int32_t E) {
    if (TAB == TAB_GLOBAL) return P.otab[E];
    if (TAB == TAB_LDS_DENSE) return ((const float *)sm)[E];
    const int32_t nw = (P.n_cat + 31) >> 5;
    const uint32_t w = sm[E >> 5];
    const uint32_t m = 1u << (E & 31);
    return (w & m) ? ((const float *)(sm + 2 * nw + 1))[sm[nw + (E >> 5)] + __popc(w & (m - 1u))]
                   : 0.0f;
}

// Occurrence view of a primary-uncertainty layer (one wavefront per trial):
// the per-event occurrence losses of the layer's table, in stored order.  The
// table sits in LDS as for the YLT pass (16-wavefront blocks sharing a copy):
// read from global memory, its 64 scattered lookups per chunk load the L2
// with a request per lane.
template <bool F64OUT, int TAB>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_pu_occ_view(PuArgs P) {
    extern __shared__ uint32_t sm[];
    pu_stage_table<TAB>(P, sm);
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t base = P.off[P.trial_begin];
    for (int64_t t = wid; t < P.trial_count; t += nwv) {
        const int64_t a = P.off[P.trial_begin + t], b = P.off[P.trial_begin + t + 1];
        double cs = 0.0, ca = 0.0;
        for (int64_t c = a; c < b; c += 64) {
            const int64_t j = c + lane;
            const bool valid = j < b;
            const double o =
                valid ? (double)pu_look<TAB>(P, sm, __builtin_nontemporal_load(P.ev + j)) : 0.0;
            occ_chunk<F64OUT>(o, valid, j - base, P.layer, P.occ_view, P.occ_stride, P.agg_r,
                              P.agg_l, &cs, &ca, P.status, P.trial_begin + t);
        }
    }
}

// A 16-byte load of the event-id stream, marked non-temporal: every id is read
// once, so it should not displace the cached tables (11 % faster for the
// primary-uncertainty pass, 0.76 -> 0.67 ms at the full shape).
__device__ __forceinline__ int4 ld_stream(const int4 *p) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    const i32x4 g = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(p));
    return make_int4(g.x, g.y, g.z, g.w);
}

// One wavefront per trial (persistent grid-stride over trials).  With the
// table in LDS a block is 16 wavefronts sharing one copy, two blocks per CU
// (32 wavefronts: the LDS copy per wavefront is what limited occupancy);
// with the table in global memory blocks are 4 wavefronts.  Event ids are
// streamed with 16-byte loads (after a scalar head that reaches 16-byte
// alignment), four loads in flight per lane.
template <int MODE, bool F64OUT, int TAB>
__device__ __forceinline__ void pu_trials(const PuArgs &P) {
    extern __shared__ uint32_t sm[];
    pu_stage_table<TAB>(P, sm);
    auto look = [&](int32_t E) -> float { return pu_look<TAB>(P, sm, E); };
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t t = wid; t < P.trial_count; t += nwv) {
        const int64_t a = P.off[P.trial_begin + t], b = P.off[P.trial_begin + t + 1];
        const int64_t n = b - a;
        Acc<MODE> acc;
        // the four losses of one 16-byte load: compensated summation adds
        // their pairwise sum (error within 2 ulp of the group, so the trial's
        // error stays a few ulp of its total whatever its length) at a
        // quarter of the per-element cost; the other modes add them one by one
        auto add4 = [&](const int4 q) {
            if (MODE == ARA_SUM_KAHAN32) {
                acc.add((look(q.x) + look(q.y)) + (look(q.z) + look(q.w)));
            } else {
                acc.add(look(q.x)); acc.add(look(q.y)); acc.add(look(q.z)); acc.add(look(q.w));
            }
        };
        // int32 elements up to the next 16-byte boundary of the event-id stream
        int64_t head = (int64_t)(((16u - ((uint32_t)(uintptr_t)(P.ev + a) & 15u)) & 15u) >> 2);
        if (head > n) head = n;
        if (lane < head) acc.add(look(P.ev[a + lane]));
        const int4 *v4 = (const int4 *)(P.ev + a + head);
        const int64_t n4 = (n - head) >> 2;
        for (int64_t i = lane; i < n4; i += 4 * 64) {
            const bool h1 = i + 64 < n4, h2 = i + 128 < n4, h3 = i + 192 < n4;
            const int4 q0 = ld_stream(v4 + i);
            int4 q1 = make_int4(0, 0, 0, 0), q2 = q1, q3 = q1;
            if (h1) q1 = ld_stream(v4 + i + 64);
            if (h2) q2 = ld_stream(v4 + i + 128);
            if (h3) q3 = ld_stream(v4 + i + 192);
            add4(q0);
            if (h1) add4(q1);
            if (h2) add4(q2);
            if (h3) add4(q3);
        }
        const int64_t done = head + 4 * n4;
        if (lane < n - done) acc.add(look(P.ev[a + done + lane]));
        const double S = acc.total();
        if (lane == 0) {
            double Y;
            if (MODE == ARA_SUM_F64) Y = clampd_terms(S, (double)P.agg_r, (double)P.agg_l);
            else Y = (double)clampf_terms((float)S, P.agg_r, P.agg_l);
            if (F64OUT) {
                if (P.ylt_layers) ((double *)P.ylt_layers)[(int64_t)P.layer * P.trial_count + t] = Y;
                if (P.ylt_pf) {
                    double *p = (double *)P.ylt_pf + t;
                    *p = P.accumulate_pf ? *p + Y : Y;
                }
            } else {
                if (P.ylt_layers)
                    ((float *)P.ylt_layers)[(int64_t)P.layer * P.trial_count + t] = (float)Y;
                if (P.ylt_pf) {
                    float *p = (float *)P.ylt_pf + t;
                    *p = P.accumulate_pf ? *p + (float)Y : (float)Y;
                }
            }
        }
    }
}

// Table in LDS: 16 wavefronts per block, 8 per SIMD (two blocks per CU).
template <int MODE, bool F64OUT, int TAB>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_ara_pu(PuArgs P) {
    pu_trials<MODE, F64OUT, TAB>(P);
}

// Table in global memory (catalogues too large for LDS): 4 wavefronts per block.
template <int MODE, bool F64OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_ara_pu_global(PuArgs P) {
    pu_trials<MODE, F64OUT, TAB_GLOBAL>(P);
}

// ---------------------------------------------------------------------------
// secondary uncertainty
// ---------------------------------------------------------------------------
// LDS per wavefront: X[kSeg] floats + Q[kQCap] pairs = 4 KB, so LDS allows 40
// waves per CU and the register budget sets the occupancy (7 per SIMD,
// measured best on the full-shape workload against 5, 6 and 8)
constexpr int kSeg = 512;         // occurrences per LDS segment
constexpr int kQCap = 256;        // hit queue (power of two)
#define ARA_SU_OCCUPANCY __attribute__((amdgpu_waves_per_eu(7, 7)))
// A layer's ELT records are staged in LDS when it has at most this many ELTs
// (1 KB more per wavefront, still within the occupancy above); the draw then
// needs one global load (the row) before its Philox key is known.
constexpr int kEltLds = 64;
constexpr int kQMask = kQCap - 1;
constexpr int kPerLane = (kQCap - kWave) / kWave;   // hits a lane appends per sub-step

struct SuArgs {
    const int64_t *off;
    const int32_t *ev;
    int64_t trial_begin, trial_count;
    const LayerDev *layers;
    int32_t n_layers;
    const EltDev *elts;
    const uint32_t *evoff;
    const RowQ *rowq;
    const RowF *rowf;
    const float *row_mean;
    const float *row_cfrac;
    const uint32_t *row_meta;
    const double *row_lnb;
    float tail_band;
    void *ylt_layers;
    void *ylt_pf;
    int64_t *hits;
    uint64_t *hit_chk;
    Status *status;
    int32_t *redo;            // trials (relative index) handed to the FP64-capable pass
    uint32_t *redo_count;
    int32_t f64_iters;        // step limit of the FP64 quantile
    const float *shape_tab;   // the portfolio's shape tables ([layer][kShapeSlots][kShapeStride])
    const uint32_t *row_shape;   // per row: 1 + its shape slot, or 0 (the diagnostic pass)
    void *occ_view;           // occurrence view, written by the DIAG and OCC instantiations
    int64_t occ_stride;
};

// The draws of a hit as 24-bit grid integers: jI keyed (k, i, elt_id, 0),
// jC keyed (k, i, 0, 1); only those the row's flags need are drawn.
// The two uniforms of a hit on the 2^-24 grid (j such that u = j 2^-24):
// jI for the independent part, jC for the correlated part, drawn only when
// the row needs them.  Occurrence keying: (k, i, elt_id, 0) and (k, i, 0, 1);
// paper keying (section 3.1's z_(Prog,E) and z_(E)): (k, i, program, 2) and
// (E, 0, 0, 3).
__device__ __forceinline__ void draw_j(uint32_t flags, int32_t keying, uint32_t k, uint32_t i,
                                       uint32_t elt_id, uint32_t program, uint32_t event,
                                       const PhiloxKeys &keys, uint32_t *jI, uint32_t *jC) {
    const bool paper = keying == ARA_KEYING_PAPER;
    const uint4 cI = paper ? make_uint4(k, i, program, 2u) : make_uint4(k, i, elt_id, 0u);
    const uint4 cC = paper ? make_uint4(event, 0u, 0u, 3u) : make_uint4(k, i, 0u, 1u);
    *jI = (flags & ROW_CONLY) ? 0u : u24(philox10_x0(cI, keys));
    *jC = (flags & (ROW_CONLY | ROW_CORR)) ? u24(philox10_x0(cC, keys)) : 0u;
}

// z and 1 - z of a hit (section 3.2).  A pure independent or correlated draw
// is an exact grid value u = j 2^-24 (and 1 - u is exact too); the mixed case
// maps both uniforms through Phi^-1 (= -sqrt(2) erfcinv(2u), taken on the side
// of the smaller tail so the argument is exact), mixes, and maps back with
// Phi(v) and Phi(-v).
template <typename T>
__device__ __forceinline__ void hit_z(uint32_t meta, uint32_t jI, uint32_t jC, T cfrac, T *z, T *zc) {
    const T s24 = (T)5.9604644775390625e-08;
    if (!(meta & ROW_CORR)) {
        const uint32_t j = (meta & ROW_CONLY) ? jC : jI;
        *z = (T)j * s24;
        *zc = (T)(16777216u - j) * s24;
        return;
    }
    auto nq = [&](uint32_t j) {
        const T lo = (T)(j < 8388608u ? j : 16777216u - j) * ((T)2 * s24);
        const T v = (T)1.4142135623730951 * erfcinv(lo);
        return j < 8388608u ? -v : v;
    };
    const T wc = cfrac, wi = (T)1 - cfrac;
    const T v = (nq(jI) * wi + nq(jC) * wc) / sqrt(wi * wi + wc * wc);
    *z = (T)0.5 * erfc(-v * (T)0.7071067811865476);
    *zc = (T)0.5 * erfc(v * (T)0.7071067811865476);
}

// One trial of the analysis, all layers (Algorithm 1 from the layer loop
// down).  REDO = false is the lean FP32 pass: a hit that needs the FP64
// quantile (tail band, shape outside the FP32 domain, FP32 non-convergence)
// abandons the trial, which is then queued for the REDO = true pass, where
// such hits take the FP64 path in place.  Returns true when abandoned.
template <int MODE, bool F64OUT, bool DIAG, bool REDO, bool OCC = false>
__device__ __forceinline__ bool su_trial(const SuArgs &A, const PhiloxKeys &keys, int64_t t,
                                         float *X, uint2 *Q, EltDev *El) {
    const int lane = threadIdx.x;
    const int64_t ti = A.trial_begin + t;
    const uint32_t i_abs = (uint32_t)ti;
    const int64_t o0 = A.off[ti];
    const int64_t n = A.off[ti + 1] - o0;
    double pf_sum = 0.0;

    for (int l = 0; l < A.n_layers; ++l) {
        const LayerDev L = A.layers[l];
        const uint32_t *eo = A.evoff + L.evoff_base;
        const int64_t rb0 = L.row_base;
        const bool elt_lds = L.n_elts <= kEltLds;
        if (elt_lds) {
            __syncthreads();
            for (int i = lane; i < L.n_elts; i += kWave) El[i] = A.elts[L.elt_begin + i];
            __syncthreads();
        }
        Acc<MODE> acc;
        uint64_t chk = 0;
        int64_t nh = 0;
        double occ_s = 0.0, occ_a = 0.0;      // occurrence-view carries
        (void)occ_s;
        (void)occ_a;

        for (int64_t seg = 0; seg < n; seg += kSeg) {
            const int segn = (int)((n - seg) < kSeg ? (n - seg) : kSeg);
            for (int i = lane; i < segn; i += kWave) X[i] = 0.0f;
            uint32_t qh = 0, qt = 0;   // queue head / tail (wave-uniform)
            bool abandon = false;
            __syncthreads();

            // Drain cnt queue entries from head h, one hit per lane: draw,
            // invert the Beta CDF, ELT terms, accumulate into X[k].
            auto run_batch = [&](uint32_t h, int cnt) {
                __syncthreads();
                bool defer = false;
                if (lane < cnt) {
                    const uint2 e = Q[(h + lane) & kQMask];
                    const uint32_t kl = e.x, row = e.y;
                    // the row's flags and Beta parameters: one compact record in
                    // the fast passes (row indexes the paying rows), the per-row
                    // arrays in the diagnostic pass (row indexes all rows)
                    uint32_t meta, orow, shape;
                    RowQ q;
                    float cfrac;
                    if (DIAG) {
                        meta = A.row_meta[row];
                        q = A.rowq[row];
                        cfrac = A.row_cfrac[row];
                        orow = row;
                        shape = A.row_shape[row];
                    } else {
                        const RowF F = A.rowf[row];
                        meta = F.meta;
                        q.scale = F.scale;
                        orow = (uint32_t)rb0 + rowf_row(F);
                        shape = rowf_shape(F);
                        cfrac = F.cfrac;
                    }
                    // the row's shape table, when its shape has a slot
                    const float *tab =
                        shape ? A.shape_tab + ((size_t)l * kShapeSlots + (shape - 1u)) * kShapeStride
                              : nullptr;
                    if (!DIAG) {
                        // Beta parameters: the slot's (the lanes of a batch mostly share
                        // one), else the row's own
                        if (tab) {
                            const float4 h = *reinterpret_cast<const float4 *>(tab + 2 * kShapeK);
                            q.a = h.x;
                            q.b = h.y;
                            q.lnb = h.z;
                        } else if (!(meta & ROW_DET)) {
                            const RowQ r = A.rowq[orow];
                            q.a = r.a;
                            q.b = r.b;
                            q.lnb = r.lnb;
                        } else {
                            q.a = q.b = q.lnb = 0.0f;
                        }
                    }
                    const uint32_t ei = meta & 0xffffu;
                    // the layer's ELT record: an LDS read when the layer's records
                    // are staged (the global read is a different instruction, so the
                    // two are not merged into one flat load)
                    EltDev ed;
                    if (elt_lds) {
                        ed = El[ei];
                    } else {
                        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                        const u32x4 g = __builtin_nontemporal_load(
                            reinterpret_cast<const u32x4 *>(A.elts + L.elt_begin + ei));
                        ed.elt_id = g.x;
                        ed.retention = __uint_as_float(g.y);
                        ed.limit = __uint_as_float(g.z);
                        ed.share = __uint_as_float(g.w);
                    }
                    float loss = 0.0f;
                    if (meta & ROW_DET) {
                        loss = q.scale;
                    } else if (!REDO && (meta & (ROW_F64 | ROW_CORR))) {
                        // shapes outside the FP32 domain and the two-normal mix
                        // (whose special functions would inflate this pass's
                        // register budget: inlined here they spill 387
                        // registers at 7 waves per SIMD) are left to the
                        // second pass
                        defer = true;
                    } else {
                        uint32_t jI, jC;
                        const uint32_t ev =
                            L.keying == ARA_KEYING_PAPER ? (uint32_t)A.ev[o0 + seg + kl] : 0u;
                        draw_j(meta, L.keying, (uint32_t)(seg + kl), i_abs, ed.elt_id,
                               L.program_id, ev, keys, &jI, &jC);
                        float z, zc;
                        if (REDO) {
                            hit_z<float>(meta, jI, jC, cfrac, &z, &zc);
                        } else {
                            const uint32_t j = (meta & ROW_CONLY) ? jC : jI;
                            z = (float)j * 5.9604644775390625e-08f;
                            zc = (float)(16777216u - j) * 5.9604644775390625e-08f;
                        }
                        bool need64 = (meta & ROW_F64) || fminf(z, zc) < A.tail_band;
                        if (!need64) {
                            bool ok;
                            const float x = beta_quantile32(q.a, q.b, q.lnb, meta_na(meta),
                                                            meta_nb(meta), z, zc, tab, &ok);
                            if (ok) loss = q.scale * x; else need64 = true;
                        }
                        if (need64) {
                            if (REDO) {
                                double z64, zc64;
                                hit_z<double>(meta, jI, jC, (double)cfrac, &z64, &zc64);
                                bool ok;
                                const double x = beta_quantile64((double)q.a, (double)q.b,
                                                                 A.row_lnb[orow], z64, zc64,
                                                                 A.f64_iters, &ok);
                                if (!ok) report(A.status, ARA_E_NUMERIC, ti, seg + kl, ed.elt_id);
                                loss = (float)((double)q.scale * x);
                            } else {
                                defer = true;
                            }
                        }
                    }
                    if (DIAG) {
                        nh += 1;
                        chk += (uint64_t)(seg + kl + 1) * 2654435761ull + (uint64_t)ed.elt_id;
                    }
                    if (!defer) {
                        const float lp = ed.share * clampf_terms(loss, ed.retention, ed.limit);
                        atomicAdd(&X[kl], lp);
                    }
                }
                if (!REDO && __any(defer)) abandon = true;
                __syncthreads();
            };

            // The fast pass enqueues only the rows that can pay, from the
            // per-event (first record, count) pairs; the diagnostic pass
            // visits every row so it counts every non-zero lookup.  The fast
            // pass keeps its loads one chunk ahead: the next chunk's pairs
            // and the event ids of the chunk after that are in flight while
            // this chunk's hits are drawn.
            const int32_t *evs = A.ev + o0 + seg;
            const uint2 *lpairs = reinterpret_cast<const uint2 *>(A.evoff + L.live_base);
            uint2 pr_next = make_uint2(0u, 0u);
            int32_t e_after = -1;
            if (!DIAG) {
                if (lane < segn) pr_next = lpairs[evs[lane]];
                if (kWave + lane < segn) e_after = evs[kWave + lane];
            }
            for (int c = 0; c < segn && !abandon; c += kWave) {
                const int kl = c + lane;
                const bool valid = kl < segn;
                uint32_t rb = 0, cnt = 0;
                if (DIAG) {
                    if (valid) {
                        const int32_t E = evs[kl];
                        rb = eo[E];
                        cnt = eo[E + 1] - rb;
                    }
                } else {
                    rb = pr_next.x;
                    cnt = pr_next.y;                  // zero past the segment's end
                    pr_next = e_after >= 0 ? lpairs[e_after] : make_uint2(0u, 0u);
                    e_after = (c + 2 * kWave + lane < segn) ? evs[c + 2 * kWave + lane] : -1;
                }
                uint32_t done = 0;
                while (!abandon) {
                    const int take = (int)min(cnt - done, (uint32_t)kPerLane);
                    int tot;
                    const int excl = wave_excl_scan(take, &tot);
                    for (int j = 0; j < take; ++j)
                        Q[(qt + excl + j) & kQMask] =
                            make_uint2((uint32_t)kl, (uint32_t)(rb0 + rb + done + j));
                    qt += tot;
                    done += take;
                    while (qt - qh >= (uint32_t)kWave && !abandon) {
                        run_batch(qh, kWave);
                        qh += kWave;
                    }
                    if (!__any(done < cnt)) break;
                }
            }
            if (!abandon && qt != qh) run_batch(qh, (int)(qt - qh));
            if (abandon) return true;
            __syncthreads();
            for (int i = lane; i < segn; i += kWave)
                acc.add(clampf_terms(X[i], L.occ_r, L.occ_l));
            if ((DIAG || OCC) && A.occ_view) {
                const int64_t pos0 = o0 - A.off[A.trial_begin] + seg;
                for (int c = 0; c < segn; c += kWave) {
                    const int i = c + lane;
                    const bool valid = i < segn;
                    const double o = valid ? (double)clampf_terms(X[i], L.occ_r, L.occ_l) : 0.0;
                    occ_chunk<F64OUT>(o, valid, pos0 + i, l, A.occ_view, A.occ_stride, L.agg_r,
                                      L.agg_l, &occ_s, &occ_a, A.status, ti);
                }
            }
            __syncthreads();
        }

        const double S = acc.total();
        double Y;
        if (MODE == ARA_SUM_F64) Y = clampd_terms(S, (double)L.agg_r, (double)L.agg_l);
        else Y = (double)clampf_terms((float)S, L.agg_r, L.agg_l);
        if (DIAG) {
            nh = wave_sum(nh);
            chk = wave_sum(chk);
        }
        if (lane == 0) {
            if (F64OUT) {
                if (A.ylt_layers) ((double *)A.ylt_layers)[(int64_t)l * A.trial_count + t] = Y;
            } else {
                if (A.ylt_layers) ((float *)A.ylt_layers)[(int64_t)l * A.trial_count + t] = (float)Y;
            }
            if (DIAG) {
                if (A.hits) A.hits[(int64_t)l * A.trial_count + t] = nh;
                if (A.hit_chk) A.hit_chk[(int64_t)l * A.trial_count + t] = chk;
            }
        }
        if (F64OUT) pf_sum += Y;
        else pf_sum = (double)((float)pf_sum + (float)Y);
    }
    if (lane == 0 && A.ylt_pf) {
        if (F64OUT) ((double *)A.ylt_pf)[t] = pf_sum;
        else ((float *)A.ylt_pf)[t] = (float)pf_sum;
    }
    return false;
}

// Main pass: one wavefront (block) per trial.  DIAG: every row visited, hit
// counts and checksums (and the occurrence view when asked for); OCC: the
// lean pass that also writes the occurrence view (its per-occurrence sums
// are those of the DIAG pass: the rows it skips add +0).
template <int MODE, bool F64OUT, bool DIAG, bool OCC = false>
__global__ __launch_bounds__(64) ARA_SU_OCCUPANCY void k_ara_su(SuArgs A, PhiloxKeys keys) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    const int64_t t = blockIdx.x;
    if (t >= A.trial_count) return;
    if (su_trial<MODE, F64OUT, DIAG, false, OCC>(A, keys, t, X, Q, El) && threadIdx.x == 0)
        A.redo[atomicAdd(A.redo_count, 1u)] = (int32_t)t;
}

// FP64-capable pass over the trials the main pass handed over; the count is
// read on the device, so no host round trip is needed between the passes.
template <int MODE, bool F64OUT, bool DIAG, bool OCC>
__device__ __forceinline__ void su_redo_loop(const SuArgs &A, const PhiloxKeys &keys, float *X,
                                             uint2 *Q, EltDev *El) {
    // the list holds at most one entry per trial of the run; an entry outside
    // the run (scratch shared by runs that overlapped, against the contract)
    // is reported instead of followed
    const uint32_t cnt = *A.redo_count;
    const uint32_t n = cnt < (uint32_t)A.trial_count ? cnt : (uint32_t)A.trial_count;
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const int32_t t = A.redo[r];
        if (t < 0 || (int64_t)t >= A.trial_count) {
            if (threadIdx.x == 0) report(A.status, ARA_E_INVALID_ARG, r, t, A.trial_count);
            continue;
        }
        su_trial<MODE, F64OUT, DIAG, true, OCC>(A, keys, (int64_t)t, X, Q, El);
    }
}

template <int MODE, bool F64OUT, bool DIAG, bool OCC = false>
__global__ __launch_bounds__(64) void k_ara_su_redo(SuArgs A, PhiloxKeys keys) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    su_redo_loop<MODE, F64OUT, DIAG, OCC>(A, keys, X, Q, El);
}

// The same pass held to 4 wavefronts per SIMD (128 registers, spilling the
// rest): for portfolios whose handed-over draws are FP64 quantiles (shapes
// outside the FP32 domain, capped sigma) four resident wavefronts hide more
// of the FP64 latency than one unspilled one; with two-normal-mix rows the
// FP32 special functions of the mix spill too and the one-wavefront form
// above is faster (both measured on the full shape).
template <int MODE, bool F64OUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_ara_su_redo4(
    SuArgs A, PhiloxKeys keys) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    su_redo_loop<MODE, F64OUT, false, false>(A, keys, X, Q, El);
}

// ---------------------------------------------------------------------------
// batched portfolios: one persistent launch over (trial tile, portfolio)
// work items, trial-major so the portfolios of one tile run close together
// and share that tile's event ids from cache; an atomic counter hands out the
// items (load balance across portfolios of very different cost)
// ---------------------------------------------------------------------------
__global__ void k_batch_reset(unsigned long long *counter, uint32_t *redo_count) {
    *counter = 0ull;
    *redo_count = 0u;
}

__global__ void k_reset_u32(uint32_t *p) { *p = 0u; }

__device__ __forceinline__ void batch_view(const BatchArgs &B, int p, SuArgs &A, PhiloxKeys &keys) {
    const BatchPf &P = B.pfs[p];
    A.off = B.off;
    A.ev = B.ev;
    A.trial_begin = P.trial_begin;
    A.trial_count = P.trial_count;
    A.layers = P.layers;
    A.n_layers = P.n_layers;
    A.elts = P.elts;
    A.evoff = P.evoff;
    A.rowq = P.rowq;
    A.rowf = P.rowf;
    A.row_mean = P.row_mean;
    A.row_cfrac = P.row_cfrac;
    A.row_meta = P.row_meta;
    A.row_lnb = P.row_lnb;
    A.tail_band = B.tail_band;
    A.ylt_layers = P.ylt_layers;
    A.ylt_pf = P.ylt_pf;
    A.hits = nullptr;
    A.hit_chk = nullptr;
    A.status = B.status;
    A.redo = nullptr;
    A.redo_count = nullptr;
    A.f64_iters = kF64QuantileIters;
    A.shape_tab = P.shape_tab;
    A.row_shape = nullptr;
    A.occ_view = nullptr;
    A.occ_stride = 0;
    keys.k0 = P.k0;
    keys.k1 = P.k1;
}

// One work item of a batch: a tile of B.tile trials of one portfolio.  The
// item index is wave-uniform; the portfolio and tile are derived from it
// (trial-major: tile-then-portfolio; portfolio-major: each portfolio's block
// of items in turn).
template <int MODE, bool F64OUT>
__device__ __forceinline__ void batch_item(const BatchArgs &B, unsigned long long item, float *X,
                                           uint2 *Q, EltDev *El) {
    int64_t tile;
    int p;
    if (B.trial_major) {
        tile = (int64_t)(item / (unsigned long long)B.n_pf);
        p = (int)(item % (unsigned long long)B.n_pf);
    } else {
        // the portfolio whose block of work items holds this item
        int lo_p = 0, hi_p = B.n_pf - 1;
        while (lo_p < hi_p) {
            const int mid = (lo_p + hi_p + 1) >> 1;
            if ((unsigned long long)B.pfs[mid].tile_base <= item) lo_p = mid; else hi_p = mid - 1;
        }
        p = lo_p;
        tile = (int64_t)item - B.pfs[p].tile_base;
    }
    // wave-uniform by construction; said explicitly so the portfolio's
    // pointers are read with scalar loads into scalar registers
    p = __builtin_amdgcn_readfirstlane(p);
    tile = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(tile >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)tile));
    SuArgs A;
    PhiloxKeys keys;
    batch_view(B, p, A, keys);
    const int64_t t0 = tile * B.tile;
    const int64_t t1 = (t0 + B.tile) < A.trial_count ? (t0 + B.tile) : A.trial_count;
    for (int64_t t = t0; t < t1; ++t)
        if (su_trial<MODE, F64OUT, false, false>(A, keys, t, X, Q, El) && threadIdx.x == 0)
            B.redo[atomicAdd(B.redo_count, 1u)] = ((unsigned long long)p << 32) | (uint64_t)t;
}

// Persistent form: grid-wide loop over work items taken from an atomic
// counter (waves_per_cu wavefronts per CU stay resident).
template <int MODE, bool F64OUT>
__global__ __launch_bounds__(64) void k_ara_batch(BatchArgs B) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    const unsigned long long n_items = (unsigned long long)B.n_items;
    while (true) {
        unsigned long long item = 0;
        if (threadIdx.x == 0) item = atomicAdd(B.counter, 1ull);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)item);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(item >> 32));
        item = ((unsigned long long)hi << 32) | lo;
        if (item >= n_items) break;
        batch_item<MODE, F64OUT>(B, item, X, Q, El);
    }
}

// One workgroup per work item: the dispatcher hands the items out in index
// order as wavefronts retire, and a wavefront keeps no state across items,
// so the kernel runs at the single-portfolio kernel's occupancy.
template <int MODE, bool F64OUT>
__global__ __launch_bounds__(64) ARA_SU_OCCUPANCY void k_ara_batch_items(BatchArgs B) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    const unsigned long long item = blockIdx.x;
    if (item >= (unsigned long long)B.n_items) return;
    batch_item<MODE, F64OUT>(B, item, X, Q, El);
}

template <int MODE, bool F64OUT>
__device__ __forceinline__ void batch_redo_loop(const BatchArgs &B, float *X, uint2 *Q, EltDev *El) {
    const uint32_t n = *B.redo_count;
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const unsigned long long e = B.redo[r];
        const int p = (int)(e >> 32);
        const int64_t t = (int64_t)(e & 0xffffffffull);
        if (p >= B.n_pf || t >= B.pfs[p].trial_count) {     // see k_ara_su_redo
            if (threadIdx.x == 0) report(B.status, ARA_E_INVALID_ARG, r, p, t);
            continue;
        }
        SuArgs A;
        PhiloxKeys keys;
        batch_view(B, p, A, keys);
        su_trial<MODE, F64OUT, false, true>(A, keys, t, X, Q, El);
    }
}

template <int MODE, bool F64OUT>
__global__ __launch_bounds__(64) void k_ara_batch_redo(BatchArgs B) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    batch_redo_loop<MODE, F64OUT>(B, X, Q, El);
}

// the batch's second pass in the register budget of k_ara_su_redo4
template <int MODE, bool F64OUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_ara_batch_redo4(
    BatchArgs B) {
    __shared__ float X[kSeg];
    __shared__ uint2 Q[kQCap];
    __shared__ EltDev El[kEltLds];
    batch_redo_loop<MODE, F64OUT>(B, X, Q, El);
}

// ---------------------------------------------------------------------------
// diagnostics
// ---------------------------------------------------------------------------
__global__ void k_debug_philox(int64_t n, const uint32_t *__restrict__ ctr, PhiloxKeys keys,
                               uint32_t *__restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint4 c = make_uint4(ctr[4 * j], ctr[4 * j + 1], ctr[4 * j + 2], ctr[4 * j + 3]);
        const uint4 r = philox10(c, keys);
        out[4 * j] = r.x;
        out[4 * j + 1] = r.y;
        out[4 * j + 2] = r.z;
        out[4 * j + 3] = r.w;
        if (philox10_x0(c, keys) != r.x) out[4 * j] = ~r.x;   // both forms must agree
    }
}

// tab: a shape table built for every entry's (a, b) (one shape), or null
__global__ __launch_bounds__(64) void k_debug_quantile(int64_t n, const float *__restrict__ a,
                                                       const float *__restrict__ b,
                                                       const double *__restrict__ z,
                                                       const double *__restrict__ zc, float tail,
                                                       const float *__restrict__ tab,
                                                       float *__restrict__ x,
                                                       int32_t *__restrict__ path) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float A = a[j], B = b[j];
    const float zf = (float)z[j], zcf = (float)zc[j];
    const bool shape_ok = A >= kF32MinShape && B >= kF32MinShape && A <= kF32MaxShape &&
                          B <= kF32MaxShape;
    bool use64 = !shape_ok || fminf(zf, zcf) < tail;
    const double lnb = lgamma((double)A) + lgamma((double)B) - lgamma((double)A + (double)B);
    float r = 0.0f;
    if (!use64) {
        const int na = cf_terms((double)A, (double)B), nb = cf_terms((double)B, (double)A);
        if (na == 0 || nb == 0) use64 = true;
        else {
            bool ok;
            r = beta_quantile32(A, B, (float)(lnb * 1.4426950408889634), na, nb, zf, zcf, tab,
                                &ok);
            if (!ok) use64 = true;
        }
    }
    if (use64) {
        bool ok;
        r = (float)beta_quantile64((double)A, (double)B, lnb, z[j], zc[j], kF64QuantileIters, &ok);
        if (!ok) r = __builtin_nanf("");
    }
    x[j] = r;
    if (path) path[j] = use64 ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_validate_yet(const int64_t *off, const int32_t *ev, const float *times,
                               int64_t n_trials, int32_t n_cat, Status *st,
                               unsigned long long *max_len, hipStream_t s) {
    // a resident grid (8 blocks of 4 wavefronts per CU of the largest part)
    // that strides over the trials: one atomic per wavefront for the longest
    // trial, not one per trial on a single address
    const int g = grid_for(n_trials, 4, 2048);
    hipLaunchKernelGGL(k_validate_yet, dim3(g), dim3(256), 0, s, off, ev, times, n_trials, n_cat,
                       st, max_len);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_check_rows(const RawRow *raw, int64_t n, int32_t n_cat, int32_t su, Status *st,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, raw, n, n_cat, su, st);
    return hipGetLastError();
}

hipError_t launch_fit_rows(const RawRow *raw, int64_t n, int32_t su, RowFit *fit, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_fit_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, raw, n, su, fit);
    return hipGetLastError();
}

hipError_t launch_build_layer(const RawRow *raw, const RowFit *fit, const int64_t *elt_row_off,
                              const EltDev *elts,
                              LayerDev *d_layer, const LayerDev &h_layer, int32_t n_cat, int32_t su,
                              int32_t *dat, uint32_t *evoff, uint32_t *liveoff, RowQ *rowq,
                              RowF *rowf, float *row_mean,
                              float *row_cfrac, uint32_t *row_meta, double *row_lnb, float *otab,
                              Status *st, hipStream_t s) {
    const int64_t nd = (int64_t)h_layer.n_elts * n_cat;
    hipError_t e = launch_fill_i32(dat, nd > 0 ? nd : 1, -1, s);
    if (e != hipSuccess) return e;
    if (h_layer.n_rows > 0)
        hipLaunchKernelGGL(k_dat_scatter, dim3(grid_for(h_layer.n_rows, 256)), dim3(256), 0, s,
                           raw, elt_row_off, h_layer.elt_begin, h_layer.n_elts, n_cat, dat, st);
    uint32_t *eo = evoff + h_layer.evoff_base;
    hipLaunchKernelGGL(k_ev_count, dim3(grid_for((int64_t)n_cat + 1, 256)), dim3(256), 0, s, dat,
                       raw, elt_row_off, elts, h_layer.elt_begin, h_layer.n_elts, n_cat, su, eo,
                       liveoff);
    hipLaunchKernelGGL(k_scan_excl_u32, dim3(1), dim3(1024), 0, s, eo, (int64_t)n_cat + 1);
    hipLaunchKernelGGL(k_scan_excl_u32, dim3(1), dim3(1024), 0, s, liveoff, (int64_t)n_cat + 1);
    hipLaunchKernelGGL(k_ev_fill, dim3(grid_for(n_cat, 256)), dim3(256), 0, s, dat, raw, fit,
                       elt_row_off, elts, d_layer, n_cat, su, eo, evoff + h_layer.live_base,
                       liveoff, rowq, rowf, row_mean, row_cfrac, row_meta, row_lnb, otab);
    return hipGetLastError();
}

hipError_t launch_build_sparse(const float *otab, int32_t n_cat, uint32_t *bits, uint32_t *rank,
                               float *vals, LayerDev *d_layer, hipStream_t s) {
    const int32_t nw = (n_cat + 31) >> 5;
    hipLaunchKernelGGL(k_sp_bits, dim3(grid_for((int64_t)nw + 1, 256)), dim3(256), 0, s, otab, n_cat,
                       bits, rank);
    hipLaunchKernelGGL(k_scan_excl_u32, dim3(1), dim3(1024), 0, s, rank, (int64_t)nw + 1);
    hipLaunchKernelGGL(k_sp_vals, dim3(grid_for(nw, 256)), dim3(256), 0, s, otab, n_cat, bits, rank,
                       vals, d_layer);
    return hipGetLastError();
}

template <int MODE, bool F64OUT>
static hipError_t pu_dispatch(const PuLaunch &p, hipStream_t s) {
    PuArgs A;
    A.off = p.off; A.ev = p.ev; A.trial_begin = p.trial_begin; A.trial_count = p.trial_count;
    A.otab = p.otab; A.sp_bits = p.sp_bits; A.sp_rank = p.sp_rank; A.sp_vals = p.sp_vals;
    A.nnz = p.nnz; A.n_cat = p.n_cat; A.agg_r = p.agg_r; A.agg_l = p.agg_l; A.layer = p.layer;
    A.ylt_layers = p.ylt_layers; A.ylt_pf = p.ylt_pf; A.accumulate_pf = p.accumulate_pf;
    A.occ_view = p.occ_view; A.occ_stride = p.occ_stride; A.status = p.status;
    const size_t nw = ((size_t)p.n_cat + 31) / 32;
    const size_t dense = (size_t)p.n_cat * sizeof(float);
    const size_t sparse = (2 * nw + 1 + (size_t)p.nnz) * sizeof(uint32_t);
    // p.grid counts blocks of 16 wavefronts (two per CU at most)
    const dim3 g(p.grid), b(1024);
    if (p.occ_view) {
        if (dense <= 32 * 1024)
            hipLaunchKernelGGL((k_pu_occ_view<F64OUT, TAB_LDS_DENSE>), g, b, dense, s, A);
        else if (sparse <= 60 * 1024)
            hipLaunchKernelGGL((k_pu_occ_view<F64OUT, TAB_LDS_SPARSE>), g, b, sparse, s, A);
        else
            hipLaunchKernelGGL((k_pu_occ_view<F64OUT, TAB_GLOBAL>), dim3(p.grid * 4), dim3(256), 0,
                               s, A);
    }
    if (dense <= 32 * 1024) {
        hipLaunchKernelGGL((k_ara_pu<MODE, F64OUT, TAB_LDS_DENSE>), g, b, dense, s, A);
    } else if (sparse <= 60 * 1024) {
        hipLaunchKernelGGL((k_ara_pu<MODE, F64OUT, TAB_LDS_SPARSE>), g, b, sparse, s, A);
    } else {
        const int64_t g4 = (p.trial_count + 3) / 4 < (int64_t)p.grid * 8 ? (p.trial_count + 3) / 4
                                                                         : (int64_t)p.grid * 8;
        hipLaunchKernelGGL((k_ara_pu_global<MODE, F64OUT>), dim3((unsigned)g4), dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_pu(const PuLaunch &p, int mode, bool f64out, hipStream_t s) {
    if (p.trial_count <= 0) return hipSuccess;
    if (mode == ARA_SUM_NAIVE32) return f64out ? pu_dispatch<ARA_SUM_NAIVE32, true>(p, s)
                                               : pu_dispatch<ARA_SUM_NAIVE32, false>(p, s);
    if (mode == ARA_SUM_KAHAN32) return f64out ? pu_dispatch<ARA_SUM_KAHAN32, true>(p, s)
                                               : pu_dispatch<ARA_SUM_KAHAN32, false>(p, s);
    return f64out ? pu_dispatch<ARA_SUM_F64, true>(p, s) : pu_dispatch<ARA_SUM_F64, false>(p, s);
}

template <int MODE, bool F64OUT>
static hipError_t su_dispatch2(const SuLaunch &p, hipStream_t s) {
    SuArgs A;
    A.off = p.off; A.ev = p.ev; A.trial_begin = p.trial_begin; A.trial_count = p.trial_count;
    A.layers = p.layers; A.n_layers = p.n_layers; A.elts = p.elts; A.evoff = p.evoff;
    A.rowq = p.rowq; A.rowf = p.rowf; A.row_mean = p.row_mean; A.row_cfrac = p.row_cfrac;
    A.row_meta = p.row_meta;
    A.row_lnb = p.row_lnb;
    A.tail_band = p.tail_band; A.ylt_layers = p.ylt_layers; A.ylt_pf = p.ylt_pf;
    A.hits = p.hits; A.hit_chk = p.hit_chk; A.status = p.status;
    A.redo = p.redo; A.redo_count = p.redo_count; A.f64_iters = p.f64_iters;
    A.shape_tab = p.shape_tab; A.row_shape = p.row_shape;
    A.occ_view = p.occ_view; A.occ_stride = p.occ_stride;
    const PhiloxKeys keys = philox_keys(p.seed);
    // a kernel, not hipMemsetAsync, so the sequence can be captured in a graph
    hipLaunchKernelGGL(k_reset_u32, dim3(1), dim3(1), 0, s, p.redo_count);
    const dim3 g((unsigned)p.trial_count), gr((unsigned)p.redo_grid);
    if (p.hits || p.hit_chk) {
        hipLaunchKernelGGL((k_ara_su<MODE, F64OUT, true>), g, dim3(64), 0, s, A, keys);
        hipLaunchKernelGGL((k_ara_su_redo<MODE, F64OUT, true>), gr, dim3(64), 0, s, A, keys);
    } else if (p.occ_view) {
        hipLaunchKernelGGL((k_ara_su<MODE, F64OUT, false, true>), g, dim3(64), 0, s, A, keys);
        hipLaunchKernelGGL((k_ara_su_redo<MODE, F64OUT, false, true>), gr, dim3(64), 0, s, A, keys);
    } else {
        hipLaunchKernelGGL((k_ara_su<MODE, F64OUT, false>), g, dim3(64), 0, s, A, keys);
        if (p.redo_w4)
            hipLaunchKernelGGL((k_ara_su_redo4<MODE, F64OUT>), gr, dim3(64), 0, s, A, keys);
        else
            hipLaunchKernelGGL((k_ara_su_redo<MODE, F64OUT, false>), gr, dim3(64), 0, s, A, keys);
    }
    return hipGetLastError();
}

hipError_t launch_scan_excl_u32(uint32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_excl_u32, dim3(1), dim3(1024), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_su(const SuLaunch &p, int mode, bool f64out, hipStream_t s) {
    if (p.trial_count <= 0) return hipSuccess;
    if (mode == ARA_SUM_NAIVE32) return f64out ? su_dispatch2<ARA_SUM_NAIVE32, true>(p, s)
                                               : su_dispatch2<ARA_SUM_NAIVE32, false>(p, s);
    if (mode == ARA_SUM_KAHAN32) return f64out ? su_dispatch2<ARA_SUM_KAHAN32, true>(p, s)
                                               : su_dispatch2<ARA_SUM_KAHAN32, false>(p, s);
    return f64out ? su_dispatch2<ARA_SUM_F64, true>(p, s) : su_dispatch2<ARA_SUM_F64, false>(p, s);
}

// grid <= 0: one workgroup per work item; otherwise the persistent form with
// that many workgroups.
template <int MODE, bool F64OUT>
static void batch_dispatch(const BatchArgs &B, int grid, int redo_grid, bool redo_w4,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, B.counter, B.redo_count);
    if (grid <= 0)
        hipLaunchKernelGGL((k_ara_batch_items<MODE, F64OUT>), dim3((unsigned)B.n_items), dim3(64),
                           0, s, B);
    else
        hipLaunchKernelGGL((k_ara_batch<MODE, F64OUT>), dim3(grid), dim3(64), 0, s, B);
    if (redo_w4)
        hipLaunchKernelGGL((k_ara_batch_redo4<MODE, F64OUT>), dim3(redo_grid), dim3(64), 0, s, B);
    else
        hipLaunchKernelGGL((k_ara_batch_redo<MODE, F64OUT>), dim3(redo_grid), dim3(64), 0, s, B);
}

hipError_t launch_batch(const BatchArgs &B, int mode, bool f64out, int grid, int redo_grid,
                        bool redo_w4, hipStream_t s) {
    if (B.n_items <= 0 || B.n_pf <= 0) return hipSuccess;
    if (mode == ARA_SUM_NAIVE32) {
        if (f64out) batch_dispatch<ARA_SUM_NAIVE32, true>(B, grid, redo_grid, redo_w4, s);
        else batch_dispatch<ARA_SUM_NAIVE32, false>(B, grid, redo_grid, redo_w4, s);
    } else if (mode == ARA_SUM_KAHAN32) {
        if (f64out) batch_dispatch<ARA_SUM_KAHAN32, true>(B, grid, redo_grid, redo_w4, s);
        else batch_dispatch<ARA_SUM_KAHAN32, false>(B, grid, redo_grid, redo_w4, s);
    } else {
        if (f64out) batch_dispatch<ARA_SUM_F64, true>(B, grid, redo_grid, redo_w4, s);
        else batch_dispatch<ARA_SUM_F64, false>(B, grid, redo_grid, redo_w4, s);
    }
    return hipGetLastError();
}

hipError_t launch_debug_philox(int64_t n, const uint32_t *ctr, uint64_t key, uint32_t *out,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_philox, dim3(grid_for(n, 256)), dim3(256), 0, s, n, ctr,
                       philox_keys(key), out);
    return hipGetLastError();
}

hipError_t launch_debug_quantile(int64_t n, const float *a, const float *b, const double *z,
                                 const double *zc, float tail, const float *tab, float *x,
                                 int32_t *path, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_quantile, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n, a, b,
                       z, zc, tail, tab, x, path);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shape tables
// ---------------------------------------------------------------------------
// The distinct Beta shapes of one layer's paying rows on the FP32 quantile
// path into kShapeSlots slots, by a rule that depends on the rows alone (so
// every load of a portfolio gives every row the same path): among the
// layer's first kShapeScan paying rows, each thread lists the first distinct
// shapes of its contiguous chunk in row order and thread 0 merges the lists
// in chunk order until the slots are full (one block per layer; keys
// [kShapeSlots] receives the slots, 0 = unused).  k_shape_assign then gives
// every paying row 1 + its slot, or 0, in its compact record and in the
// per-row array.
constexpr uint32_t kShapeScan = 4096;

__device__ __forceinline__ bool shape_eligible(const RowF &F) {
    return !(F.meta & (ROW_DET | ROW_F64));
}
__device__ __forceinline__ unsigned long long shape_key(const RowQ &q) {
    return ((unsigned long long)__float_as_uint(q.a) << 32) | __float_as_uint(q.b);
}

__global__ __launch_bounds__(256) void k_shape_collect(const RowF *__restrict__ rowf,
                                                       const RowQ *__restrict__ rowq,
                                                       int64_t row_base,
                                                       const uint32_t *__restrict__ liveoff,
                                                       int32_t n_cat,
                                                       unsigned long long *__restrict__ keys) {
    __shared__ unsigned long long loc[256][kShapeSlots];
    __shared__ int locn[256];
    __shared__ unsigned long long slot[kShapeSlots];
    const int tid = threadIdx.x;
    const uint32_t n = min(liveoff[n_cat], kShapeScan);
    const uint32_t per = (n + 255u) / 256u;
    const uint32_t lo = (uint32_t)tid * per, hi = min(n, lo + per);
    int m = 0;
    for (uint32_t i = lo; i < hi && m < kShapeSlots; ++i) {
        const RowF F = rowf[row_base + i];
        if (!shape_eligible(F)) continue;
        const unsigned long long key = shape_key(rowq[row_base + rowf_row(F)]);
        bool seen = false;
        for (int q = 0; q < m; ++q) seen = seen || loc[tid][q] == key;
        if (!seen) loc[tid][m++] = key;
    }
    locn[tid] = m;
    __syncthreads();
    if (tid == 0) {
        int ns = 0;
        for (int t = 0; t < 256 && ns < kShapeSlots; ++t)
            for (int q = 0; q < locn[t] && ns < kShapeSlots; ++q) {
                const unsigned long long key = loc[t][q];
                bool seen = false;
                for (int k = 0; k < ns; ++k) seen = seen || slot[k] == key;
                if (!seen) slot[ns++] = key;
            }
        for (int k = ns; k < kShapeSlots; ++k) slot[k] = 0ull;
    }
    __syncthreads();
    if (tid < kShapeSlots) keys[tid] = slot[tid];
}

__global__ __launch_bounds__(256) void k_shape_assign(RowF *__restrict__ rowf,
                                                      const RowQ *__restrict__ rowq, int64_t row_base,
                                                      const uint32_t *__restrict__ liveoff,
                                                      int32_t n_cat,
                                                      const unsigned long long *__restrict__ keys,
                                                      uint32_t *__restrict__ row_shape) {
    __shared__ unsigned long long slot[kShapeSlots];
    if (threadIdx.x < kShapeSlots) slot[threadIdx.x] = keys[threadIdx.x];
    __syncthreads();
    const uint32_t n = liveoff[n_cat];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        RowF &F = rowf[row_base + i];
        uint32_t sh = 0;
        if (shape_eligible(F)) {
            const unsigned long long key = shape_key(rowq[row_base + rowf_row(F)]);
            for (int k = 0; k < kShapeSlots; ++k)
                if (slot[k] == key) {
                    sh = (uint32_t)k + 1u;
                    break;
                }
        }
        F.rs = (F.rs & ~31u) | sh;
        row_shape[row_base + rowf_row(F)] = sh;
    }
}

// The tables of the used slots: one block per slot, one thread per point.
__global__ __launch_bounds__(2 * kShapeK) void k_shape_tables(const unsigned long long *__restrict__ keys,
                                                              float *__restrict__ tab) {
    const unsigned long long key = keys[blockIdx.x];
    if (key == 0ull) return;
    const double a = (double)__uint_as_float((uint32_t)(key >> 32));
    const double b = (double)__uint_as_float((uint32_t)key);
    const double lnb = lgamma(a) + lgamma(b) - lgamma(a + b);
    const int upper = threadIdx.x / kShapeK, k = threadIdx.x % kShapeK;
    float *slot = tab + (size_t)blockIdx.x * kShapeStride;
    slot[threadIdx.x] = shape_table_logit(a, b, lnb, upper, k);
    // the Beta parameters of the slot's rows, as the row fit computes them
    if (threadIdx.x == 0)
        *reinterpret_cast<float4 *>(slot + 2 * kShapeK) =
            make_float4((float)a, (float)b, (float)(lnb * 1.4426950408889634), 0.0f);
}

hipError_t launch_shape_collect(RowF *rowf, const RowQ *rowq, int64_t row_base, int64_t n_rows,
                                const uint32_t *liveoff, int32_t n_cat, uint32_t *row_shape,
                                unsigned long long *keys, hipStream_t s) {
    hipLaunchKernelGGL(k_shape_collect, dim3(1), dim3(256), 0, s, rowf, rowq, row_base, liveoff,
                       n_cat, keys);
    // a grid over the layer's rows (the paying ones are a prefix of them)
    hipLaunchKernelGGL(k_shape_assign, dim3(grid_for(n_rows > 0 ? n_rows : 1, 256, 1024)),
                       dim3(256), 0, s, rowf, rowq, row_base, liveoff, n_cat, keys, row_shape);
    return hipGetLastError();
}

hipError_t launch_shape_tables(const unsigned long long *keys, int64_t n_slots, float *tab,
                               hipStream_t s) {
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shape_tables, dim3((unsigned)n_slots), dim3(2 * kShapeK), 0, s, keys,
                       tab);
    return hipGetLastError();
}

}  // namespace ara
