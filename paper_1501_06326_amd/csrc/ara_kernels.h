// ara_kernels.h -- host-side launch interface of the ARA kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara_internal.h"

namespace ara {

struct PuLaunch {
    const int64_t *off;
    const int32_t *ev;
    int64_t trial_begin, trial_count;
    const float *otab;          // the layer's per-event occurrence losses [n_cat]
    const uint32_t *sp_bits;    // its sparse form: bitmap [nw], rank [nw + 1], values [nnz]
    const uint32_t *sp_rank;
    const float *sp_vals;
    int32_t nnz;
    int32_t n_cat;
    float agg_r, agg_l;
    int32_t layer;
    void *ylt_layers;
    void *ylt_pf;
    int32_t accumulate_pf;      // 0: ylt_pf = Y, 1: ylt_pf += Y
    int grid;
    void *occ_view;             // optional occurrence view (see ara_run_opts)
    int64_t occ_stride;
    Status *status;
};

struct SuLaunch {
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
    uint64_t seed;
    float tail_band;
    void *ylt_layers;
    void *ylt_pf;
    int64_t *hits;
    uint64_t *hit_chk;
    Status *status;
    int32_t *redo;            // [trial_count] scratch: trials handed to the FP64-capable pass
    uint32_t *redo_count;     // scratch counter
    int redo_grid;            // blocks of the second pass
    int redo_w4;              // second pass at 4 wavefronts per SIMD (FP64-quantile rows, no mix)
    int32_t f64_iters;        // step limit of the FP64 quantile
    const float *shape_tab;   // shape tables [layer][kShapeSlots][kShapeStride]
    const uint32_t *row_shape;   // per row: 1 + shape slot, or 0
    void *occ_view;           // optional occurrence view (see ara_run_opts)
    int64_t occ_stride;
};

// One portfolio of a batched run (device array of these).
struct BatchPf {
    const LayerDev *layers;
    const EltDev *elts;
    const uint32_t *evoff;
    const RowQ *rowq;
    const RowF *rowf;
    const float *row_mean;
    const float *row_cfrac;
    const uint32_t *row_meta;
    const double *row_lnb;
    const float *shape_tab;    // shape tables [layer][kShapeSlots][kShapeStride]
    void *ylt_layers;
    void *ylt_pf;
    uint32_t k0, k1;           // Philox key (the portfolio's seed)
    int32_t n_layers;
    int32_t pad;
    int64_t trial_begin, trial_count;   // the portfolio's trial range
    int64_t tile_base;                  // its first work item (trial-major off)
};

struct BatchArgs {
    const int64_t *off;
    const int32_t *ev;
    int64_t trial_begin, trial_count;
    const BatchPf *pfs;
    int32_t n_pf;
    int32_t tile;                       // trials per work item
    float tail_band;
    int32_t trial_major;                // 1: one common range, items (tile, portfolio)
    int64_t n_items;                    // work items
    unsigned long long *counter;        // work-item counter
    unsigned long long *redo;           // (portfolio << 32 | trial) handed to the FP64 pass
    uint32_t *redo_count;
    Status *status;
};

hipError_t launch_validate_yet(const int64_t *off, const int32_t *ev, const float *times,
                               int64_t n_trials, int32_t n_cat, Status *st,
                               unsigned long long *max_len, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_check_rows(const RawRow *raw, int64_t n, int32_t n_cat, int32_t su, Status *st,
                             hipStream_t s);
hipError_t launch_fit_rows(const RawRow *raw, int64_t n, int32_t su, RowFit *fit, hipStream_t s);
hipError_t launch_build_layer(const RawRow *raw, const RowFit *fit, const int64_t *elt_row_off,
                              const EltDev *elts,
                              LayerDev *d_layer, const LayerDev &h_layer, int32_t n_cat, int32_t su,
                              int32_t *dat, uint32_t *evoff, uint32_t *liveoff, RowQ *rowq,
                              RowF *rowf, float *row_mean,
                              float *row_cfrac, uint32_t *row_meta, double *row_lnb, float *otab,
                              Status *st, hipStream_t s);
hipError_t launch_pu(const PuLaunch &p, int mode, bool f64out, hipStream_t s);
hipError_t launch_build_sparse(const float *otab, int32_t n_cat, uint32_t *bits, uint32_t *rank,
                               float *vals, LayerDev *d_layer, hipStream_t s);
hipError_t launch_su(const SuLaunch &p, int mode, bool f64out, hipStream_t s);
hipError_t launch_batch(const BatchArgs &B, int mode, bool f64out, int grid, int redo_grid,
                        bool redo_w4,
                        hipStream_t s);
// exclusive prefix sum of p[0, n) in place (one block; also used by the
// exceedance-curve sort for its digit counts)
hipError_t launch_scan_excl_u32(uint32_t *p, int64_t n, hipStream_t s);
hipError_t launch_debug_philox(int64_t n, const uint32_t *ctr, uint64_t key, uint32_t *out,
                               hipStream_t s);
hipError_t launch_debug_quantile(int64_t n, const float *a, const float *b, const double *z,
                                 const double *zc, float tail, const float *tab, float *x,
                                 int32_t *path, hipStream_t s);
// shape tables: the distinct shapes of one layer's paying rows into keys
// [kShapeSlots] (rows get their slot), then the tables of n_slots slots
hipError_t launch_shape_collect(RowF *rowf, const RowQ *rowq, int64_t row_base, int64_t n_rows,
                                const uint32_t *liveoff, int32_t n_cat, uint32_t *row_shape,
                                unsigned long long *keys, hipStream_t s);
hipError_t launch_shape_tables(const unsigned long long *keys, int64_t n_slots, float *tab,
                               hipStream_t s);

// measurement probes (ara_probe.hip)
hipError_t launch_probe_stream(const void *src, int64_t n16, uint32_t *sink, int n_cu,
                               hipStream_t s);
hipError_t launch_probe_valu(int kind, int blocks, int32_t iters, float *out, hipStream_t s);
hipError_t launch_probe_row_consts(float a, float b, int32_t *d_out, hipStream_t s);
hipError_t launch_probe_draws(int64_t n, uint64_t seed, uint32_t elt_id, float a, float b,
                              float lnb2, int32_t na, int32_t nb, const float *tab, float *x,
                              hipStream_t s);

// PML / TVaR and the exceedance-probability curve (ara_select.hip)
size_t pml_scratch_bytes(int64_t n);
size_t ep_scratch_bytes(int64_t n, int32_t dtype);
hipError_t launch_ep_curve(const void *ylt, int32_t dtype, int64_t n, void *sorted,
                           double *tail_mean, void *scratch, hipStream_t s);
hipError_t launch_pml_tvar(const void *ylt, int32_t dtype, int64_t n, const int64_t *ks, int32_t n_rp,
                           void *scratch, double *d_out /* [2 * n_rp]: pml, tvar */, hipStream_t s);

}  // namespace ara
