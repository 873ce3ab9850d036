// ara_internal.h -- device data layout shared by the host runtime and the
// kernels of the ARA library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara.h"

namespace ara {

// Row metadata word: bits 0-15 ELT index in the layer, bits 16-19 flags,
// bits 20-25 / 26-31 the continued-fraction terms of the (a, b) / (b, a)
// branches of the FP32 quantile.
enum : uint32_t {
    ROW_DET = 1u << 16,    // loss = mean (sigma = 0 or secondary uncertainty off)
    ROW_F64 = 1u << 17,    // shape outside the FP32 quantile's domain: FP64 path
    ROW_CORR = 1u << 18,   // sigma_I > 0 and sigma_C > 0: mix two normals (section 3.2)
    ROW_CONLY = 1u << 19,  // sigma_I = 0, sigma_C > 0: z = u_C
    ROW_FLAGS = 0xFu << 16,
};
__host__ __device__ inline int meta_na(uint32_t m) { return (int)((m >> 20) & 63u); }
__host__ __device__ inline int meta_nb(uint32_t m) { return (int)((m >> 26) & 63u); }

// Per-layer record in device memory.
struct LayerDev {
    float occ_r, occ_l, agg_r, agg_l;   // layer terms (FP32; limits may be +inf)
    int32_t elt_begin;                   // first ELT (index into EltDev[])
    int32_t n_elts;
    int64_t row_base;                    // first row of the layer in the row arrays
    int64_t evoff_base;                  // first entry of the layer's ev_off[n_cat + 1]
    int64_t otab_base;                   // first entry of the layer's otab[n_cat] (PU), or -1
    uint32_t flags;                      // OR of the row flags of the layer
    int32_t n_rows;
    int32_t nnz;                         // non-zero entries of otab (PU)
    uint32_t program_id;                 // keys z_(Prog,E) under ARA_KEYING_PAPER
    int32_t keying;                      // ARA_KEYING_* of the portfolio
    int32_t pad;
    int64_t live_base;                   // even index of the layer's (ev_off[E], rows of E
                                         // that can pay) pairs in the ev_off array
};

// Per-ELT record: id (keys the draws) and ELT financial terms.
struct EltDev {
    uint32_t elt_id;
    float retention, limit, share;
};

// Per-row secondary-uncertainty constants, event-major inside each layer:
// {max_l, alpha, beta, ln B(alpha, beta)} with ln B evaluated in FP64 at the
// FP32 alpha, beta (so the FP32 and FP64 quantiles solve the same equation).
struct RowQ {
    float scale, a, b, lnb;
};

// Compact record of a row that can pay, read by the fast passes with one
// 16-byte load: the layer's such rows are contiguous, event-major.  rs packs
// the index of the same row in the layer's per-row arrays (bits 5-31, so a
// layer holds fewer than kRowFMaxRows rows) and 1 + the slot of the row's
// Beta shape among the layer's shape tables, or 0 when it has none (bits
// 0-4); cfrac is the two-normal mix weight.  A row with a slot takes its
// Beta parameters (alpha, beta, log2 B(alpha, beta)) from the slot, which
// holds exactly the values of its rows (they are functions of the shape
// alone); a row without one reads them from the per-row arrays.
struct __attribute__((aligned(16))) RowF {
    float scale;
    uint32_t meta;
    uint32_t rs;
    float cfrac;
};
constexpr int64_t kRowFMaxRows = (int64_t)1 << 27;
__host__ __device__ inline uint32_t rowf_row(const RowF &F) { return F.rs >> 5; }
__host__ __device__ inline uint32_t rowf_shape(const RowF &F) { return F.rs & 31u; }

// Raw host rows staged on the device for the build kernels.
struct RawRow {
    int32_t event;
    float mean, sigma_i, sigma_c, max_loss;
};

// The Beta fit of one raw row (build staging, indexed like the raw rows).
struct RowFit {
    RowQ q;
    uint32_t flags;
    float cfrac;
    double lnb;
};

// Context-owned device status words.
struct Status {
    int32_t code;          // 0 or an ara_status of the first failure
    int32_t pad;
    int64_t where[3];      // first failing (trial, occurrence, elt_id) or row index
};

constexpr int kWave = 64;

// Shapes the FP32 quantile covers (its error stays below ~1e-6 of the root
// there); others take the FP64 path.
constexpr float kF32MinShape = 1.0f;
constexpr float kF32MaxShape = 32.0f;

// Step limit of the FP64 quantile's bracketed iteration; a draw that has not
// converged by then is reported as ARA_E_NUMERIC.
constexpr int kF64QuantileIters = 400;

// Beta shapes shared by many rows.  Each layer has kShapeSlots slots; the
// first distinct (alpha, beta) pairs of its rows on the FP32 quantile path
// take one each.  A slot holds, for each half of the draw grid (z <= 1/2 and
// z > 1/2, with p = min(z, 1 - z)), the logit log(x / (1 - x)) of the
// quantile x at kShapeK points evenly spaced in t = sqrt(-2 ln p) over
// [sqrt(2 ln 2), sqrt(48 ln 2)] (p from 1/2 down to 2^-24): linear
// interpolation in t starts the quantile within ~2.2e-4 of its root for every
// shape of the FP32 domain, close enough for a single Halley step.
constexpr int kShapeSlots = 16;
constexpr int kShapeK = 128;
// floats per slot: the two halves, then (alpha, beta, log2 B(alpha, beta), 0)
constexpr int kShapeStride = 2 * kShapeK + 4;
constexpr double kShapeTLo = 1.1774100225154747;   // sqrt(2 ln 2)
constexpr double kShapeTHi = 5.768107546403532;    // sqrt(48 ln 2)

}  // namespace ara

// Host-side handle definitions (not visible to the C-ABI).
struct ara_yet {
    ara_context *ctx;
    int64_t n_trials;
    int32_t n_catalogue;
    const int64_t *d_off;
    const int32_t *d_ev;
    const float *d_times;
    int64_t n_occ;
    int64_t max_trial_len;
};

struct ara_portfolio {
    ara_context *ctx;
    int32_t n_catalogue;
    int32_t n_layers;
    int32_t n_elts;
    int64_t n_rows;
    uint64_t seed;
    int32_t su_enabled;
    int32_t max_layer_elts;
    uint32_t all_flags;
    ara::LayerDev *d_layers;
    ara::EltDev *d_elts;
    uint32_t *d_evoff;
    ara::RowQ *d_rowq;
    ara::RowF *d_rowf;
    float *d_row_mean;
    float *d_row_cfrac;
    uint32_t *d_row_meta;
    double *d_row_lnb;
    uint32_t *d_row_shape;     // per row: 1 + its shape slot, or 0
    unsigned long long *d_shape_keys;   // [layer][kShapeSlots]: (alpha, beta) bits, 0 = unused
    float *d_shape_tab;        // [layer][kShapeSlots][kShapeStride]
    float *d_otab;
    uint32_t *d_sp_bits;       // per layer [nw]: bitmap of the non-zero otab entries
    uint32_t *d_sp_rank;       // per layer [nw + 1]: set bits before each word
    float *d_sp_vals;          // per layer [n_cat]: the non-zero otab values, in event order
    void *d_workspace;
    size_t workspace_bytes;
    ara::LayerDev *h_layers;   // host copy
};

namespace ara {
// Batched run with a trial range per portfolio (ranges[2i], ranges[2i+1]),
// portfolio-major; device-side errors go to *status (null: the context's own
// status word).  Defined with the C-ABI, used by the serving loop.
ara_status run_batch_ranges(ara_context *ctx, const ara_yet *yet, int32_t n,
                            ara_portfolio *const *pfs, const ara_run_opts *opts,
                            const ara_batch_config *cfg, void *const *ylt_l, void *const *ylt_p,
                            const int64_t *ranges, void *scratch, size_t bytes, void *stream,
                            Status *status);
// Batch scratch for n portfolios whose trial ranges add up to total_trials.
size_t batch_scratch_need(int32_t n, int64_t total_trials);
}  // namespace ara

