// ara_api.hip -- host runtime behind the C-ABI of include/ara.h: contexts,
// argument validation, the portfolio workspace layout, launches and error
// reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "ara.h"
#include "ara_internal.h"
#include "ara_kernels.h"

using namespace ara;

// Scratch of ara_run_static: the hand-over from the FP32 pass to the
// FP64-capable pass (a counter, then one trial index per trial) for up to
// ARA_STATIC_MAX_TRIALS trials, in a device array each GPU holds for the life
// of the process.  Host code reaches it only through the address
// hipGetSymbolAddress gives for the current device (static_scratch_address).
constexpr size_t kStaticScratchBytes = 256 + sizeof(int32_t) * (size_t)ARA_STATIC_MAX_TRIALS;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct ara_context {
    int device = 0;
    int n_cu = 0;
    void *d_static_scratch = nullptr;       // this device's copy of `scratch`
    std::string last_error;
    Status *d_status = nullptr;             // device status words
    unsigned long long *d_maxlen = nullptr;
    std::set<ara_yet *> yets;
    std::set<ara_portfolio *> pfs;
    std::set<ara_graph *> graphs;
};

struct ara_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kMaxRp = 256;
// 2^-24, the smallest draw on the grid: every draw takes the FP32 quantile
// (its residual is taken on the smaller side, accurate to ~1e-7 down to
// 2^-24); the FP64 path serves shapes outside the FP32 domain, sigma-capped
// rows and FP32 non-convergence.
constexpr float kDefaultTailBand = 5.9604644775390625e-08f;

size_t run_scratch_need(int64_t trial_count) {
    return 256 + ((size_t)(trial_count > 0 ? trial_count : 1) * sizeof(int32_t) + 255) / 256 * 256;
}

// The FP32 pass hands the trials it cannot finish to the FP64-capable pass
// through scratch: a counter at the start, the trial list 256 bytes in.  The
// second pass takes up to as many wavefronts as the first keeps resident
// (7 per SIMD), each looping over the list; surplus ones find it empty.
void su_scratch(const ara_context *ctx, SuLaunch *p, char *scr, const ara_run_opts &o) {
    p->redo_count = (uint32_t *)scr;
    p->redo = (int32_t *)(scr + 256);
    const int64_t resident = (int64_t)ctx->n_cu * 4 * 7;
    p->redo_grid = (int)(o.trial_count < resident ? (o.trial_count > 0 ? o.trial_count : 1)
                                                  : resident);
    if (o.debug_flags & ARA_DEBUG_QUANTILE_ONE_STEP) {
        p->tail_band = 2.0f;       // every draw takes the FP64 quantile ...
        p->f64_iters = 1;          // ... which may take one step
    } else {
        p->f64_iters = kF64QuantileIters;
    }
}

// The primary-uncertainty pass of one portfolio over trials [begin, begin +
// count): per layer, the gather-sum over the per-event occurrence-loss table
// (ara_run, and the primary-uncertainty portfolios of a batch).
hipError_t enqueue_pu(const ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                      int64_t begin, int64_t count, int32_t sum_mode, bool f64out,
                      void *ylt_layers, void *ylt_pf, void *occ_view, int64_t occ_stride,
                      Status *status, hipStream_t s);

ara_status fail(ara_context *ctx, ara_status code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

#define ARA_HIP(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), ARA_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte layout of a portfolio workspace.
struct Layout {
    size_t layers, elts, evoff, liveoff, rowq, rowf, row_mean, row_cfrac, row_meta, row_lnb,
        row_shape, shape_keys, shape_tab, otab,
        sp_bits, sp_rank,
        sp_vals, raw, rawfit, eltoff, dat, total;
    int64_t n_rows = 0;
    int32_t n_elts = 0, max_layer_elts = 0;
};

ara_status plan(ara_context *ctx, const ara_portfolio_desc *d, int32_t n_cat, Layout *L) {
    if (!d || n_cat <= 0 || d->n_layers < 0 || (d->n_layers > 0 && !d->layers))
        return fail(ctx, ARA_E_INVALID_ARG, "bad portfolio description or catalogue size");
    if (d->keying != ARA_KEYING_OCCURRENCE && d->keying != ARA_KEYING_PAPER)
        return fail(ctx, ARA_E_INVALID_ARG, "unknown keying %d", d->keying);
    int64_t rows = 0;
    int32_t ne = 0, mx = 0;
    for (int l = 0; l < d->n_layers; ++l) {
        const ara_layer_desc &ld = d->layers[l];
        if (ld.n_elts < 0 || (ld.n_elts > 0 && !ld.elts) || ld.n_elts > 65535)
            return fail(ctx, ARA_E_INVALID_ARG, "layer %d: bad ELT list", l);
        if (!(ld.occ_retention >= 0) || !(ld.agg_retention >= 0) || !(ld.occ_limit >= 0) ||
            !(ld.agg_limit >= 0) || std::isinf(ld.occ_retention) || std::isinf(ld.agg_retention))
            return fail(ctx, ARA_E_BAD_ELT_ROW, "layer %d: terms must be finite retentions >= 0 "
                                                "and limits >= 0", l);
        int64_t layer_rows = 0;
        for (int j = 0; j < ld.n_elts; ++j) {
            const ara_elt_desc &e = ld.elts[j];
            if (e.n_rows < 0 || (e.n_rows > 0 && (!e.event_ids || !e.mean)))
                return fail(ctx, ARA_E_INVALID_ARG, "layer %d ELT %d: missing rows", l, j);
            if (!(e.share >= 0.0 && e.share <= 1.0) || !(e.retention >= 0) ||
                std::isinf(e.retention) || !(e.limit >= 0))
                return fail(ctx, ARA_E_BAD_ELT_ROW, "layer %d ELT %d: share must be in [0,1], "
                                                    "retention finite >= 0, limit >= 0", l, j);
            rows += e.n_rows;
            layer_rows += e.n_rows;
        }
        if (layer_rows >= kRowFMaxRows)
            return fail(ctx, ARA_E_UNSUPPORTED, "layer %d: 2^27 or more ELT rows in one layer", l);
        ne += ld.n_elts;
        if (ld.n_elts > mx) mx = ld.n_elts;
    }
    if (rows >= ((int64_t)1 << 32) - 1)
        return fail(ctx, ARA_E_UNSUPPORTED, "more than 2^32 ELT rows in one portfolio");
    L->n_rows = rows;
    L->n_elts = ne;
    L->max_layer_elts = mx;
    const int64_t nl = d->n_layers;
    size_t o = 0;
    L->layers = o; o += align256(sizeof(LayerDev) * (nl ? nl : 1));
    L->elts = o; o += align256(sizeof(EltDev) * (ne ? ne : 1));
    // per layer ev_off[n_cat + 1]; then, from an even index, per layer the
    // pairs (ev_off[e], rows of e that can pay) [n_cat] (one 8-byte load per
    // occurrence in the fast pass)
    L->evoff = o;
    o += align256(sizeof(uint32_t) * ((size_t)nl * ((size_t)n_cat + 1) + 1 + (size_t)nl * 2 * n_cat));
    L->liveoff = o; o += align256(sizeof(uint32_t) * (size_t)nl * ((size_t)n_cat + 1));
    L->rowq = o; o += align256(sizeof(RowQ) * (size_t)(rows ? rows : 1));
    L->rowf = o; o += align256(sizeof(RowF) * (size_t)(rows ? rows : 1));
    L->row_mean = o; o += align256(sizeof(float) * (size_t)(rows ? rows : 1));
    L->row_cfrac = o; o += align256(sizeof(float) * (size_t)(rows ? rows : 1));
    L->row_meta = o; o += align256(sizeof(uint32_t) * (size_t)(rows ? rows : 1));
    L->row_lnb = o; o += align256(sizeof(double) * (size_t)(rows ? rows : 1));
    const bool su = d->su_enabled != 0;
    L->row_shape = o; o += su ? align256(sizeof(uint32_t) * (size_t)(rows ? rows : 1)) : 0;
    L->shape_keys = o; o += su ? align256(sizeof(unsigned long long) * kShapeSlots * (nl ? nl : 1)) : 0;
    L->shape_tab = o;
    o += su ? align256(sizeof(float) * kShapeStride * kShapeSlots * (size_t)(nl ? nl : 1)) : 0;
    const size_t nw = ((size_t)n_cat + 31) / 32;
    const bool pu = !d->su_enabled;
    L->otab = o; o += pu ? align256(sizeof(float) * (size_t)nl * n_cat) : 0;
    L->sp_bits = o; o += pu ? align256(sizeof(uint32_t) * (size_t)nl * nw) : 0;
    L->sp_rank = o; o += pu ? align256(sizeof(uint32_t) * (size_t)nl * (nw + 1)) : 0;
    L->sp_vals = o; o += pu ? align256(sizeof(float) * (size_t)nl * n_cat) : 0;
    L->raw = o; o += align256(sizeof(RawRow) * (size_t)(rows ? rows : 1));
    L->rawfit = o; o += align256(sizeof(RowFit) * (size_t)(rows ? rows : 1));
    L->eltoff = o; o += align256(sizeof(int64_t) * (size_t)(ne + 1));
    L->dat = o; o += align256(sizeof(int32_t) * (size_t)(mx ? mx : 1) * n_cat);
    L->total = o;
    return ARA_OK;
}

hipError_t enqueue_pu(const ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                      int64_t begin, int64_t count, int32_t sum_mode, bool f64out,
                      void *ylt_layers, void *ylt_pf, void *occ_view, int64_t occ_stride,
                      Status *status, hipStream_t s) {
    const size_t nwc = ((size_t)pf->n_catalogue + 31) / 32;
    for (int l = 0; l < pf->n_layers; ++l) {
        PuLaunch p;
        p.off = yet->d_off;
        p.ev = yet->d_ev;
        p.trial_begin = begin;
        p.trial_count = count;
        p.otab = pf->d_otab + (int64_t)l * pf->n_catalogue;
        p.sp_bits = pf->d_sp_bits + (size_t)l * nwc;
        p.sp_rank = pf->d_sp_rank + (size_t)l * (nwc + 1);
        p.sp_vals = pf->d_sp_vals + (size_t)l * pf->n_catalogue;
        p.nnz = pf->h_layers[l].nnz;
        p.n_cat = pf->n_catalogue;
        p.agg_r = pf->h_layers[l].agg_r;
        p.agg_l = pf->h_layers[l].agg_l;
        p.layer = l;
        p.ylt_layers = ylt_layers;
        p.ylt_pf = ylt_pf;
        p.accumulate_pf = l > 0;
        p.occ_view = occ_view;
        p.occ_stride = occ_stride;
        p.status = status;
        // blocks of 16 wavefronts, two resident per CU (LDS table <= 60 KB)
        const int64_t blocks = (count + 15) / 16;
        const int64_t g = blocks < (int64_t)ctx->n_cu * 2 ? blocks : (int64_t)ctx->n_cu * 2;
        p.grid = (int)(g < 1 ? 1 : g);
        const hipError_t e = launch_pu(p, sum_mode, f64out, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

ara_status check_status(ara_context *ctx, hipStream_t s, const char *what) {
    Status h;
    ARA_HIP(ctx, hipMemcpyAsync(&h, ctx->d_status, sizeof h, hipMemcpyDeviceToHost, s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    if (h.code == 0) return ARA_OK;
    ARA_HIP(ctx, hipMemsetAsync(ctx->d_status, 0, sizeof(Status), s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    switch (h.code) {
    case ARA_E_EVENT_ID_RANGE:
        return fail(ctx, h.code, "%s: event id %lld out of range (trial %lld, position %lld)", what,
                    (long long)h.where[2], (long long)h.where[0], (long long)h.where[1]);
    case ARA_E_OFFSETS_NOT_MONOTONE:
        return fail(ctx, h.code, "%s: trial offsets not monotone at trial %lld", what,
                    (long long)h.where[0]);
    case ARA_E_TIMES_UNSORTED:
        return fail(ctx, h.code, "%s: time stamps decrease in trial %lld at occurrence %lld", what,
                    (long long)h.where[0], (long long)h.where[1]);
    case ARA_E_BAD_ELT_ROW:
        return fail(ctx, h.code, "%s: bad ELT row %lld%s", what, (long long)h.where[1],
                    h.where[0] == -2 ? " (duplicate event in one ELT)" : "");
    case ARA_E_WORKSPACE_TOO_SMALL:
        return fail(ctx, h.code, "%s: occurrence view stride %lld too small (trial %lld needs "
                                 "index %lld)", what, (long long)h.where[2], (long long)h.where[0],
                    (long long)h.where[1]);
    case ARA_E_INVALID_ARG:
        return fail(ctx, h.code, "%s: hand-over entry %lld between the passes names trial %lld "
                                 "outside the run (scratch shared by runs that overlapped?)",
                    what, (long long)h.where[0], (long long)h.where[1]);
    case ARA_E_NUMERIC:
        return fail(ctx, h.code, "%s: Beta quantile did not converge (trial %lld, occurrence %lld, "
                                 "elt_id %lld)", what, (long long)h.where[0], (long long)h.where[1],
                    (long long)h.where[2]);
    default:
        return fail(ctx, h.code, "%s: device reported status %d", what, h.code);
    }
}

float to_f32_term(double v) { return std::isinf(v) ? INFINITY : (float)v; }

uint32_t fbits(float v) {
    uint32_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}

// A shape table for one (a, b) in freshly allocated device memory (the two
// diagnostics below only): key + table; the caller frees *mem.
ara_status one_shape_table(ara_context *ctx, float a, float b, hipStream_t s, void **mem,
                           float **tab) {
    *mem = nullptr;
    const size_t bytes = 256 + sizeof(float) * kShapeStride;
    ARA_HIP(ctx, hipMalloc(mem, bytes));
    const unsigned long long key = ((unsigned long long)fbits(a) << 32) | fbits(b);
    ARA_HIP(ctx, hipMemcpyAsync(*mem, &key, sizeof key, hipMemcpyHostToDevice, s));
    *tab = (float *)((char *)*mem + 256);
    ARA_HIP(ctx, launch_shape_tables((const unsigned long long *)*mem, 1, *tab, s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    return ARA_OK;
}

}  // namespace

extern "C" {

const char *ara_status_string(ara_status s) {
    switch (s) {
    case ARA_OK: return "ok";
    case ARA_E_INVALID_ARG: return "invalid argument";
    case ARA_E_NO_DEVICE: return "no such device";
    case ARA_E_HIP: return "HIP runtime error";
    case ARA_E_EVENT_ID_RANGE: return "event id out of range";
    case ARA_E_OFFSETS_NOT_MONOTONE: return "trial offsets not monotone";
    case ARA_E_TIMES_UNSORTED: return "time stamps unsorted";
    case ARA_E_BAD_ELT_ROW: return "bad ELT row";
    case ARA_E_WORKSPACE_TOO_SMALL: return "workspace too small";
    case ARA_E_NUMERIC: return "numeric failure";
    case ARA_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *ara_last_error(const ara_context *ctx) {
    return ctx ? ctx->last_error.c_str() : "no context";
}

namespace {
// The device address of `scratch` on each device, looked up once per device
// with that device current.
std::mutex g_static_mu;
void *g_static_addr[256] = {};

hipError_t static_scratch_address(int device, void **addr) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (device < 0 || device >= 256) return hipErrorInvalidDevice;
    if (!g_static_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_addr[device] = p;
    }
    *addr = g_static_addr[device];
    return hipSuccess;
}
}  // namespace

ara_status ara_create(int hip_device, ara_context **out) {
    if (!out) return ARA_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
        return ARA_E_NO_DEVICE;
    ara_context *ctx = new ara_context();
    ctx->device = hip_device;
    hipDeviceProp_t prop;
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
        delete ctx;
        return ARA_E_HIP;
    }
    ctx->n_cu = prop.multiProcessorCount;
    if (static_scratch_address(hip_device, &ctx->d_static_scratch) != hipSuccess) {
        delete ctx;
        return ARA_E_HIP;
    }
    if (hipMalloc((void **)&ctx->d_status, sizeof(Status)) != hipSuccess ||
        hipMalloc((void **)&ctx->d_maxlen, sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(ctx->d_status, 0, sizeof(Status)) != hipSuccess) {
        (void)hipFree(ctx->d_status);
        delete ctx;
        return ARA_E_HIP;
    }
    *out = ctx;
    return ARA_OK;
}

void ara_destroy(ara_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (ara_yet *y : ctx->yets) delete y;
    for (ara_portfolio *p : ctx->pfs) {
        delete[] p->h_layers;
        delete p;
    }
    for (ara_graph *g : ctx->graphs) {
        (void)hipGraphExecDestroy(g->exec);
        (void)hipGraphDestroy(g->graph);
        delete g;
    }
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->d_maxlen);
    delete ctx;
}

ara_status ara_load_yet(ara_context *ctx, int64_t n_trials, int32_t n_catalogue,
                        const int64_t *d_trial_offsets, const int32_t *d_event_ids,
                        const float *d_times, void *stream, ara_yet **out) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!out || n_trials < 0 || n_catalogue <= 0 || !d_trial_offsets ||
        n_trials > (int64_t)0xffffffff)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_load_yet: bad arguments");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, hipMemsetAsync(ctx->d_status, 0, sizeof(Status), s));
    ARA_HIP(ctx, hipMemsetAsync(ctx->d_maxlen, 0, sizeof(unsigned long long), s));
    // the occurrence count first: the event ids may be absent only when there
    // are none (the validation reads ids only inside [0, offsets[n_trials]))
    int64_t n_occ = 0;
    ARA_HIP(ctx, hipMemcpyAsync(&n_occ, d_trial_offsets + n_trials, sizeof n_occ,
                                hipMemcpyDeviceToHost, s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    if (n_occ > 0 && !d_event_ids)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_load_yet: no event ids for %lld occurrences",
                    (long long)n_occ);
    if (n_trials > 0)
        ARA_HIP(ctx, launch_validate_yet(d_trial_offsets, d_event_ids, d_times, n_trials,
                                         n_catalogue, ctx->d_status, ctx->d_maxlen, s));
    unsigned long long maxlen = 0;
    ARA_HIP(ctx, hipMemcpyAsync(&maxlen, ctx->d_maxlen, sizeof maxlen, hipMemcpyDeviceToHost, s));
    ara_status st = check_status(ctx, s, "ara_load_yet");
    if (st != ARA_OK) return st;
    if (maxlen > 0xffffffffull)
        return fail(ctx, ARA_E_UNSUPPORTED, "ara_load_yet: a trial has >= 2^32 occurrences");
    ara_yet *y = new ara_yet();
    y->ctx = ctx;
    y->n_trials = n_trials;
    y->n_catalogue = n_catalogue;
    y->d_off = d_trial_offsets;
    y->d_ev = d_event_ids;
    y->d_times = d_times;
    y->n_occ = n_occ;
    y->max_trial_len = (int64_t)maxlen;
    ctx->yets.insert(y);
    *out = y;
    return ARA_OK;
}

ara_status ara_free_yet(ara_context *ctx, ara_yet *yet) {
    if (!ctx || !yet || !ctx->yets.count(yet)) return ARA_E_INVALID_ARG;
    ctx->yets.erase(yet);
    delete yet;
    return ARA_OK;
}

ara_status ara_portfolio_workspace_size(const ara_portfolio_desc *desc, int32_t n_catalogue,
                                        size_t *bytes) {
    if (!bytes) return ARA_E_INVALID_ARG;
    Layout L;
    ara_status st = plan(nullptr, desc, n_catalogue, &L);
    if (st != ARA_OK) return st;
    *bytes = L.total;
    return ARA_OK;
}

ara_status ara_load_portfolio(ara_context *ctx, const ara_portfolio_desc *desc,
                              int32_t n_catalogue, void *d_workspace, size_t bytes, void *stream,
                              ara_portfolio **out) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!out) return fail(ctx, ARA_E_INVALID_ARG, "ara_load_portfolio: null out");
    *out = nullptr;
    Layout L;
    ara_status st = plan(ctx, desc, n_catalogue, &L);
    if (st != ARA_OK) return st;
    if (!d_workspace || bytes < L.total)
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL, "ara_load_portfolio: need %zu bytes, got %zu",
                    L.total, bytes);
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    char *w = (char *)d_workspace;

    // host staging: layer and ELT records, raw rows grouped by ELT
    const int nl = desc->n_layers;
    std::vector<LayerDev> hl(nl > 0 ? nl : 1);
    std::vector<EltDev> he(L.n_elts > 0 ? L.n_elts : 1);
    std::vector<RawRow> raw((size_t)(L.n_rows > 0 ? L.n_rows : 1));
    std::vector<int64_t> eltoff((size_t)L.n_elts + 1, 0);
    int32_t ei = 0;
    int64_t ri = 0;
    for (int l = 0; l < nl; ++l) {
        const ara_layer_desc &ld = desc->layers[l];
        LayerDev &D = hl[l];
        std::memset(&D, 0, sizeof D);
        D.occ_r = to_f32_term(ld.occ_retention);
        D.occ_l = to_f32_term(ld.occ_limit);
        D.agg_r = to_f32_term(ld.agg_retention);
        D.agg_l = to_f32_term(ld.agg_limit);
        D.elt_begin = ei;
        D.n_elts = ld.n_elts;
        D.row_base = ri;
        D.evoff_base = (int64_t)l * ((int64_t)n_catalogue + 1);
        D.live_base = (((int64_t)nl * ((int64_t)n_catalogue + 1) + 1) & ~(int64_t)1) +
                      (int64_t)l * 2 * n_catalogue;
        D.otab_base = desc->su_enabled ? -1 : (int64_t)l * n_catalogue;
        D.flags = 0;
        D.program_id = ld.program_id;
        D.keying = desc->keying;
        for (int j = 0; j < ld.n_elts; ++j, ++ei) {
            const ara_elt_desc &e = ld.elts[j];
            he[ei].elt_id = e.elt_id;
            he[ei].retention = to_f32_term(e.retention);
            he[ei].limit = to_f32_term(e.limit);
            he[ei].share = (float)e.share;
            for (int r = 0; r < e.n_rows; ++r, ++ri) {
                RawRow &R = raw[(size_t)ri];
                R.event = e.event_ids[r];
                R.mean = e.mean[r];
                R.sigma_i = e.sigma_i ? e.sigma_i[r] : 0.0f;
                R.sigma_c = e.sigma_c ? e.sigma_c[r] : 0.0f;
                R.max_loss = e.max_loss ? e.max_loss[r] : INFINITY;
            }
            eltoff[(size_t)ei + 1] = ri;
        }
        D.n_rows = (int32_t)(ri - D.row_base);
    }

    ara_portfolio *p = new ara_portfolio();
    p->ctx = ctx;
    p->n_catalogue = n_catalogue;
    p->n_layers = nl;
    p->n_elts = L.n_elts;
    p->n_rows = L.n_rows;
    p->seed = desc->seed;
    p->su_enabled = desc->su_enabled ? 1 : 0;
    p->max_layer_elts = L.max_layer_elts;
    p->d_layers = (LayerDev *)(w + L.layers);
    p->d_elts = (EltDev *)(w + L.elts);
    p->d_evoff = (uint32_t *)(w + L.evoff);
    p->d_rowq = (RowQ *)(w + L.rowq);
    p->d_rowf = (RowF *)(w + L.rowf);
    p->d_row_mean = (float *)(w + L.row_mean);
    p->d_row_cfrac = (float *)(w + L.row_cfrac);
    p->d_row_meta = (uint32_t *)(w + L.row_meta);
    p->d_row_lnb = (double *)(w + L.row_lnb);
    p->d_row_shape = desc->su_enabled ? (uint32_t *)(w + L.row_shape) : nullptr;
    p->d_shape_keys = desc->su_enabled ? (unsigned long long *)(w + L.shape_keys) : nullptr;
    p->d_shape_tab = desc->su_enabled ? (float *)(w + L.shape_tab) : nullptr;
    p->d_otab = desc->su_enabled ? nullptr : (float *)(w + L.otab);
    p->d_sp_bits = desc->su_enabled ? nullptr : (uint32_t *)(w + L.sp_bits);
    p->d_sp_rank = desc->su_enabled ? nullptr : (uint32_t *)(w + L.sp_rank);
    p->d_sp_vals = desc->su_enabled ? nullptr : (float *)(w + L.sp_vals);
    p->d_workspace = d_workspace;
    p->workspace_bytes = bytes;
    RawRow *d_raw = (RawRow *)(w + L.raw);
    int64_t *d_eltoff = (int64_t *)(w + L.eltoff);
    int32_t *d_dat = (int32_t *)(w + L.dat);

    auto cleanup = [&](ara_status code) {
        delete p;
        return code;
    };
#define ARA_HIP_P(call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return cleanup(fail(ctx, ARA_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_))); \
    } while (0)

    ARA_HIP_P(hipMemsetAsync(ctx->d_status, 0, sizeof(Status), s));
    if (nl > 0)
        ARA_HIP_P(hipMemcpyAsync(p->d_layers, hl.data(), sizeof(LayerDev) * nl,
                                 hipMemcpyHostToDevice, s));
    if (L.n_elts > 0)
        ARA_HIP_P(hipMemcpyAsync(p->d_elts, he.data(), sizeof(EltDev) * L.n_elts,
                                 hipMemcpyHostToDevice, s));
    if (L.n_rows > 0)
        ARA_HIP_P(hipMemcpyAsync(d_raw, raw.data(), sizeof(RawRow) * (size_t)L.n_rows,
                                 hipMemcpyHostToDevice, s));
    ARA_HIP_P(hipMemcpyAsync(d_eltoff, eltoff.data(), sizeof(int64_t) * eltoff.size(),
                             hipMemcpyHostToDevice, s));
    ARA_HIP_P(launch_check_rows(d_raw, L.n_rows, n_catalogue, p->su_enabled, ctx->d_status, s));
    {
        ara_status cs = check_status(ctx, s, "ara_load_portfolio");
        if (cs != ARA_OK) return cleanup(cs);
    }
    RowFit *d_fit = (RowFit *)(w + L.rawfit);
    ARA_HIP_P(launch_fit_rows(d_raw, L.n_rows, p->su_enabled, d_fit, s));
    const size_t nwc = ((size_t)n_catalogue + 31) / 32;
    if (p->su_enabled && L.n_rows > 0)
        ARA_HIP_P(launch_fill_i32((int32_t *)p->d_row_shape, L.n_rows, 0, s));
    for (int l = 0; l < nl; ++l) {
        uint32_t *liveoff_l = (uint32_t *)(w + L.liveoff) + (size_t)l * ((size_t)n_catalogue + 1);
        ARA_HIP_P(launch_build_layer(d_raw, d_fit, d_eltoff, p->d_elts, p->d_layers + l, hl[l],
                                     n_catalogue,
                                     p->su_enabled, d_dat, p->d_evoff, liveoff_l,
                                     p->d_rowq, p->d_rowf, p->d_row_mean,
                                     p->d_row_cfrac, p->d_row_meta, p->d_row_lnb, p->d_otab,
                                     ctx->d_status, s));
        if (p->su_enabled)
            ARA_HIP_P(launch_shape_collect(p->d_rowf, p->d_rowq, hl[l].row_base, hl[l].n_rows, liveoff_l,
                                           n_catalogue, p->d_row_shape,
                                           p->d_shape_keys + (size_t)l * kShapeSlots, s));
        if (!p->su_enabled)
            ARA_HIP_P(launch_build_sparse(p->d_otab + (size_t)l * n_catalogue, n_catalogue,
                                          p->d_sp_bits + (size_t)l * nwc,
                                          p->d_sp_rank + (size_t)l * (nwc + 1),
                                          p->d_sp_vals + (size_t)l * n_catalogue, p->d_layers + l, s));
    }
    if (p->su_enabled)
        ARA_HIP_P(launch_shape_tables(p->d_shape_keys, (int64_t)nl * kShapeSlots, p->d_shape_tab,
                                      s));
    p->h_layers = new LayerDev[nl > 0 ? nl : 1];
    if (nl > 0)
        ARA_HIP_P(hipMemcpyAsync(p->h_layers, p->d_layers, sizeof(LayerDev) * nl,
                                 hipMemcpyDeviceToHost, s));
    {
        ara_status cs = check_status(ctx, s, "ara_load_portfolio");
        if (cs != ARA_OK) {
            delete[] p->h_layers;
            return cleanup(cs);
        }
    }
#undef ARA_HIP_P
    p->all_flags = 0;
    for (int l = 0; l < nl; ++l) p->all_flags |= p->h_layers[l].flags;
    ctx->pfs.insert(p);
    *out = p;
    return ARA_OK;
}

ara_status ara_free_portfolio(ara_context *ctx, ara_portfolio *pf) {
    if (!ctx || !pf || !ctx->pfs.count(pf)) return ARA_E_INVALID_ARG;
    ctx->pfs.erase(pf);
    delete[] pf->h_layers;
    delete pf;
    return ARA_OK;
}

}  // extern "C"

namespace {
// ara_run and ara_run_static: the same run, with the hand-over scratch of
// the caller (opts->d_scratch) or the library's static array.
ara_status run_impl(ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                    const ara_run_opts *opts, void *d_ylt_layers, void *d_ylt_portfolio,
                    void *stream, bool static_scratch) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!yet || !pf || !ctx->yets.count(const_cast<ara_yet *>(yet)) ||
        !ctx->pfs.count(const_cast<ara_portfolio *>(pf)))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: unknown YET or portfolio handle");
    if (yet->n_catalogue != pf->n_catalogue)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: YET catalogue %d != portfolio catalogue %d",
                    yet->n_catalogue, pf->n_catalogue);
    ara_run_opts o;
    std::memset(&o, 0, sizeof o);
    o.trial_count = -1;
    if (opts) o = *opts;
    if (o.trial_count < 0) o.trial_count = yet->n_trials - o.trial_begin;
    if (o.trial_begin < 0 || o.trial_count < 0 || o.trial_begin + o.trial_count > yet->n_trials)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: trial range [%lld, +%lld) outside the YET",
                    (long long)o.trial_begin, (long long)o.trial_count);
    if (o.sum_mode < 0 || o.sum_mode > ARA_SUM_F64 || o.ylt_dtype < ARA_F32 ||
        o.ylt_dtype > ARA_F64)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: bad sum_mode or ylt_dtype");
    if (o.trial_count > 0x7fffffff)
        return fail(ctx, ARA_E_UNSUPPORTED, "ara_run: more than 2^31 trials in one run");
    if (!(o.tail_band > 0.0f)) o.tail_band = kDefaultTailBand;
    if (o.debug_flags & ~ARA_DEBUG_QUANTILE_ONE_STEP)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: unknown debug flags 0x%x", o.debug_flags);
    if (o.d_occ_view && o.occ_view_stride <= 0)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run: occurrence view without a positive stride");
    if (o.trial_count == 0 || pf->n_layers == 0) {
        hipStream_t s = (hipStream_t)stream;
        const size_t es = o.ylt_dtype == ARA_F64 ? 8 : 4;
        ARA_HIP(ctx, hipSetDevice(ctx->device));
        if (d_ylt_portfolio && o.trial_count > 0)
            ARA_HIP(ctx, hipMemsetAsync(d_ylt_portfolio, 0, es * o.trial_count, s));
        return ARA_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    const bool f64out = o.ylt_dtype == ARA_F64;
    if (!pf->su_enabled) {
        if (o.d_hits || o.d_hit_chk)
            return fail(ctx, ARA_E_UNSUPPORTED,
                        "ara_run: hit diagnostics need a portfolio with secondary uncertainty");
        ARA_HIP(ctx, enqueue_pu(ctx, yet, pf, o.trial_begin, o.trial_count, o.sum_mode, f64out,
                                d_ylt_layers, d_ylt_portfolio, o.d_occ_view, o.occ_view_stride,
                                ctx->d_status, s));
        return ARA_OK;
    }
    SuLaunch p;
    p.off = yet->d_off;
    p.ev = yet->d_ev;
    p.trial_begin = o.trial_begin;
    p.trial_count = o.trial_count;
    p.layers = pf->d_layers;
    p.n_layers = pf->n_layers;
    p.elts = pf->d_elts;
    p.evoff = pf->d_evoff;
    p.rowq = pf->d_rowq;
    p.rowf = pf->d_rowf;
    p.row_mean = pf->d_row_mean;
    p.row_cfrac = pf->d_row_cfrac;
    p.row_meta = pf->d_row_meta;
    p.row_lnb = pf->d_row_lnb;
    p.shape_tab = pf->d_shape_tab;
    p.row_shape = pf->d_row_shape;
    p.seed = pf->seed;
    p.tail_band = o.tail_band;
    p.ylt_layers = d_ylt_layers;
    p.ylt_pf = d_ylt_portfolio;
    p.hits = o.d_hits;
    p.hit_chk = o.d_hit_chk;
    p.occ_view = o.d_occ_view;
    p.occ_stride = o.occ_view_stride;
    p.status = ctx->d_status;
    p.redo_w4 = (pf->all_flags & ROW_F64) && !(pf->all_flags & ROW_CORR);
    const size_t need = run_scratch_need(o.trial_count);
    char *scr = (char *)o.d_scratch;
    if (static_scratch) {
        scr = (char *)ctx->d_static_scratch;
    } else if (!scr || o.scratch_bytes < need) {
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL,
                    "ara_run: secondary uncertainty needs %zu bytes of scratch (opts->d_scratch)",
                    need);
    }
    su_scratch(ctx, &p, scr, o);
    ARA_HIP(ctx, launch_su(p, o.sum_mode, f64out, s));
    return ARA_OK;
}
}  // namespace

extern "C" {

ara_status ara_run(ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                   const ara_run_opts *opts, void *d_ylt_layers, void *d_ylt_portfolio,
                   void *stream) {
    return run_impl(ctx, yet, pf, opts, d_ylt_layers, d_ylt_portfolio, stream, false);
}

ara_status ara_run_static(ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                          const ara_run_opts *opts, void *d_ylt_layers, void *d_ylt_portfolio,
                          void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!yet || !ctx->yets.count(const_cast<ara_yet *>(yet)))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run_static: unknown YET handle");
    int64_t count = -1, begin = 0;
    if (opts) {
        count = opts->trial_count;
        begin = opts->trial_begin;
    }
    if (count < 0) count = yet->n_trials - begin;
    if (count > (int64_t)ARA_STATIC_MAX_TRIALS)
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL,
                    "ara_run_static: %lld trials exceed the static scratch (at most %d per call)",
                    (long long)count, (int)ARA_STATIC_MAX_TRIALS);
    return run_impl(ctx, yet, pf, opts, d_ylt_layers, d_ylt_portfolio, stream, true);
}

ara_status ara_run_scratch_size(int64_t trial_count, size_t *bytes) {
    if (!bytes || trial_count < 0) return ARA_E_INVALID_ARG;
    *bytes = run_scratch_need(trial_count);
    return ARA_OK;
}

ara_status ara_sync_status(ara_context *ctx, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    return check_status(ctx, (hipStream_t)stream, "ara_run");
}

ara_status ara_pml_tvar_scratch_size(int64_t n, size_t *bytes) {
    if (!bytes || n < 0) return ARA_E_INVALID_ARG;
    *bytes = align256(pml_scratch_bytes(n)) + align256(sizeof(double) * 2 * kMaxRp);
    return ARA_OK;
}

ara_status ara_pml_tvar(ara_context *ctx, const void *d_ylt, int32_t ylt_dtype, int64_t n,
                        const double *return_periods, int32_t n_rp, double *pml_out,
                        double *tvar_out, void *d_scratch, size_t scratch_bytes, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!d_ylt || n <= 0 || !return_periods || n_rp <= 0 || n_rp > kMaxRp || !pml_out ||
        !tvar_out || (ylt_dtype != ARA_F32 && ylt_dtype != ARA_F64))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_pml_tvar: bad arguments");
    size_t need = 0;
    ara_pml_tvar_scratch_size(n, &need);
    if (!d_scratch || scratch_bytes < need)
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL, "ara_pml_tvar: need %zu scratch bytes", need);
    std::vector<int64_t> ks(n_rp);
    for (int r = 0; r < n_rp; ++r) {
        const double rp = return_periods[r];
        if (!(rp > 0.0)) return fail(ctx, ARA_E_INVALID_ARG, "ara_pml_tvar: return period <= 0");
        double kk = std::floor((double)n / rp);
        int64_t k = kk < 1.0 ? 1 : (kk > (double)n ? n : (int64_t)kk);
        ks[r] = k;
    }
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    double *d_out = (double *)((char *)d_scratch + align256(pml_scratch_bytes(n)));
    ARA_HIP(ctx, launch_pml_tvar(d_ylt, ylt_dtype, n, ks.data(), n_rp, d_scratch, d_out, s));
    std::vector<double> h(2 * (size_t)n_rp);
    ARA_HIP(ctx, hipMemcpyAsync(h.data(), d_out, sizeof(double) * 2 * n_rp, hipMemcpyDeviceToHost, s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    for (int r = 0; r < n_rp; ++r) {
        pml_out[r] = h[r];
        tvar_out[r] = h[(size_t)n_rp + r];
    }
    return ARA_OK;
}

ara_status ara_ep_curve_scratch_size(int64_t n, int32_t ylt_dtype, size_t *bytes) {
    if (!bytes || n < 0 || (ylt_dtype != ARA_F32 && ylt_dtype != ARA_F64)) return ARA_E_INVALID_ARG;
    *bytes = ep_scratch_bytes(n, ylt_dtype);
    return ARA_OK;
}

ara_status ara_ep_curve(ara_context *ctx, const void *d_ylt, int32_t ylt_dtype, int64_t n,
                        void *d_sorted, double *d_tail_mean, void *d_scratch,
                        size_t scratch_bytes, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!d_ylt || !d_sorted)) || d_sorted == d_ylt ||
        (ylt_dtype != ARA_F32 && ylt_dtype != ARA_F64) || n > 0xffffffffll)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_ep_curve: bad arguments");
    if (n == 0) return ARA_OK;
    const size_t need = ep_scratch_bytes(n, ylt_dtype);
    if (!d_scratch || scratch_bytes < need)
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL, "ara_ep_curve: need %zu scratch bytes", need);
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, launch_ep_curve(d_ylt, ylt_dtype, n, d_sorted, d_tail_mean, d_scratch,
                                 (hipStream_t)stream));
    return ARA_OK;
}

// ---- batched portfolios ----------------------------------------------------
namespace {

size_t batch_pf_off() { return 256; }
size_t batch_redo_off(int32_t n) { return align256(batch_pf_off() + sizeof(BatchPf) * (size_t)n); }
// the redo list holds at most one entry per (portfolio, trial) of the batch
size_t batch_need(int32_t n, int64_t total_trials) {
    return batch_redo_off(n) + sizeof(unsigned long long) * (size_t)(total_trials > 0 ? total_trials : 1);
}

// A primary-uncertainty portfolio of a batch: it runs the per-event table
// pass of ara_run after the batched launch, on the same stream.
struct PuItem {
    const ara_portfolio *pf;
    int64_t begin, count;
    void *ylt_layers, *ylt_pf;
};

struct BatchPlan {
    BatchArgs B;
    int grid, redo_grid, mode;
    bool f64out;
    bool redo_w4;       // second pass at 4 wavefronts per SIMD (see k_ara_su_redo4)
    std::vector<PuItem> pu;
};

// Validate a batch and upload its portfolio table.  ranges: per portfolio
// (trial_begin, trial_count), or null for opts' common range.  Trial-major
// order needs the common range.
ara_status prep_batch_ranges(ara_context *ctx, const ara_yet *yet, int32_t n,
                             ara_portfolio *const *pfs, const ara_run_opts *opts,
                             const ara_batch_config *cfg, void *const *ylt_l, void *const *ylt_p,
                             const int64_t *ranges, void *scratch, size_t bytes, hipStream_t s,
                             Status *status, BatchPlan *plan) {
    if (!yet || !ctx->yets.count(const_cast<ara_yet *>(yet)) || n <= 0 || !pfs)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: bad YET or portfolio list");
    ara_run_opts o;
    std::memset(&o, 0, sizeof o);
    o.trial_count = -1;
    if (opts) o = *opts;
    if (o.trial_count < 0) o.trial_count = yet->n_trials - o.trial_begin;
    if (o.sum_mode < 0 || o.sum_mode > ARA_SUM_F64 || o.ylt_dtype < ARA_F32 ||
        o.ylt_dtype > ARA_F64)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: bad sum_mode or ylt_dtype");
    if (o.d_hits || o.d_hit_chk || o.d_occ_view)
        return fail(ctx, ARA_E_UNSUPPORTED,
                    "ara_run_batch: hit diagnostics and the occurrence view are per-portfolio only");
    if (!(o.tail_band > 0.0f)) o.tail_band = kDefaultTailBand;
    ara_batch_config c = {1, 0, ARA_BATCH_TRIAL_MAJOR};
    if (cfg) {
        c = *cfg;
    } else {
        for (int32_t i = 0; i < n; ++i)
            if (pfs && pfs[i] && pfs[i]->su_enabled) c.order = ARA_BATCH_PORTFOLIO_MAJOR;
    }
    if (c.trial_tile < 1 || c.waves_per_cu < 0 ||
        (c.order != ARA_BATCH_PORTFOLIO_MAJOR && c.order != ARA_BATCH_TRIAL_MAJOR))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: bad batch configuration");
    if (ranges && c.order == ARA_BATCH_TRIAL_MAJOR)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: trial-major order needs one trial range");
    int64_t total = 0, items = 0;
    std::vector<BatchPf> h;
    uint32_t su_flags = 0;     // OR of the row flags of the batch's SU portfolios
    h.reserve((size_t)n);
    plan->pu.clear();
    for (int32_t i = 0; i < n; ++i) {
        const int64_t tb = ranges ? ranges[2 * i] : o.trial_begin;
        const int64_t tc = ranges ? ranges[2 * i + 1] : o.trial_count;
        if (tb < 0 || tc < 0 || tb + tc > yet->n_trials || tc > 0x7fffffff)
            return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: trial range of portfolio %d outside "
                                                "the YET", i);
        const ara_portfolio *p = pfs[i];
        if (!p || !ctx->pfs.count(const_cast<ara_portfolio *>(p)))
            return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: unknown portfolio %d", i);
        if (p->n_catalogue != yet->n_catalogue)
            return fail(ctx, ARA_E_INVALID_ARG, "ara_run_batch: portfolio %d catalogue mismatch", i);
        if (!p->su_enabled) {
            plan->pu.push_back({p, tb, tc, ylt_l ? ylt_l[i] : nullptr, ylt_p ? ylt_p[i] : nullptr});
            continue;
        }
        su_flags |= p->all_flags;
        h.emplace_back();
        BatchPf &b = h.back();
        b.layers = p->d_layers;
        b.elts = p->d_elts;
        b.evoff = p->d_evoff;
        b.rowq = p->d_rowq;
        b.rowf = p->d_rowf;
        b.row_mean = p->d_row_mean;
        b.row_cfrac = p->d_row_cfrac;
        b.row_meta = p->d_row_meta;
        b.row_lnb = p->d_row_lnb;
        b.shape_tab = p->d_shape_tab;
        b.ylt_layers = ylt_l ? ylt_l[i] : nullptr;
        b.ylt_pf = ylt_p ? ylt_p[i] : nullptr;
        b.k0 = (uint32_t)p->seed;
        b.k1 = (uint32_t)(p->seed >> 32);
        b.n_layers = p->n_layers;
        b.pad = 0;
        b.trial_begin = tb;
        b.trial_count = tc;
        b.tile_base = items;
        items += (tc + c.trial_tile - 1) / c.trial_tile;
        total += tc;
    }
    const size_t need = batch_need(n, total);
    if (!scratch || bytes < need)
        return fail(ctx, ARA_E_WORKSPACE_TOO_SMALL, "ara_run_batch: need %zu scratch bytes", need);
    char *sc = (char *)scratch;
    if (!h.empty())
        ARA_HIP(ctx, hipMemcpyAsync(sc + batch_pf_off(), h.data(), sizeof(BatchPf) * h.size(),
                                    hipMemcpyHostToDevice, s));
    const int32_t n_su = (int32_t)h.size();
    BatchArgs &B = plan->B;
    B.off = yet->d_off;
    B.ev = yet->d_ev;
    const bool trial_major = c.order == ARA_BATCH_TRIAL_MAJOR;
    B.trial_begin = trial_major ? o.trial_begin : 0;
    B.trial_count = trial_major ? o.trial_count : 0;
    B.pfs = (const BatchPf *)(sc + batch_pf_off());
    B.n_pf = n_su;
    B.tile = c.trial_tile;
    B.tail_band = o.tail_band;
    B.trial_major = trial_major ? 1 : 0;
    B.n_items = trial_major ? ((o.trial_count + c.trial_tile - 1) / c.trial_tile) * (int64_t)n_su
                            : items;
    B.counter = (unsigned long long *)sc;
    B.redo_count = (uint32_t *)(sc + 8);
    B.redo = (unsigned long long *)(sc + batch_redo_off(n));
    B.status = status ? status : ctx->d_status;
    if (c.waves_per_cu == 0 && B.n_items > 0x7fffffffll)
        return fail(ctx, ARA_E_UNSUPPORTED, "ara_run_batch: more than 2^31 work items for the "
                                            "one-workgroup-per-item form; use waves_per_cu > 0");
    plan->grid = ctx->n_cu * c.waves_per_cu;           // 0: one workgroup per item
    plan->redo_w4 = (su_flags & ROW_F64) && !(su_flags & ROW_CORR);
    plan->redo_grid = ctx->n_cu * 4 * (plan->redo_w4 ? 4 : 1);
    plan->mode = o.sum_mode;
    plan->f64out = o.ylt_dtype == ARA_F64;
    return ARA_OK;
}

// The batched launch of a plan's secondary-uncertainty portfolios, then the
// per-event table pass of each primary-uncertainty one, all on stream s.
hipError_t launch_plan(const ara_context *ctx, const ara_yet *yet, const BatchPlan &plan,
                       hipStream_t s) {
    hipError_t e = launch_batch(plan.B, plan.mode, plan.f64out, plan.grid, plan.redo_grid, plan.redo_w4, s);
    for (size_t k = 0; k < plan.pu.size() && e == hipSuccess; ++k) {
        const PuItem &u = plan.pu[k];
        if (u.count > 0)
            e = enqueue_pu(ctx, yet, u.pf, u.begin, u.count, plan.mode, plan.f64out, u.ylt_layers,
                           u.ylt_pf, nullptr, 0, plan.B.status, s);
    }
    return e;
}

ara_status prep_batch(ara_context *ctx, const ara_yet *yet, int32_t n, ara_portfolio *const *pfs,
                      const ara_run_opts *opts, const ara_batch_config *cfg,
                      void *const *ylt_l, void *const *ylt_p, void *scratch, size_t bytes,
                      hipStream_t s, BatchPlan *plan) {
    return prep_batch_ranges(ctx, yet, n, pfs, opts, cfg, ylt_l, ylt_p, nullptr, scratch, bytes, s,
                             nullptr, plan);
}

}  // namespace

ara_status ara_batch_scratch_size(int32_t n_portfolios, int64_t trial_count, size_t *bytes) {
    if (!bytes || n_portfolios <= 0 || trial_count < 0) return ARA_E_INVALID_ARG;
    *bytes = batch_need(n_portfolios, (int64_t)n_portfolios * trial_count);
    return ARA_OK;
}

ara_status ara_run_batch(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                         ara_portfolio *const *pfs, const ara_run_opts *opts,
                         const ara_batch_config *cfg, void *const *d_ylt_layers,
                         void *const *d_ylt_portfolio, void *d_scratch, size_t scratch_bytes,
                         void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    BatchPlan plan;
    ara_status st = prep_batch(ctx, yet, n_portfolios, pfs, opts, cfg, d_ylt_layers,
                               d_ylt_portfolio, d_scratch, scratch_bytes, s, &plan);
    if (st != ARA_OK) return st;
    ARA_HIP(ctx, launch_plan(ctx, yet, plan, s));
    return ARA_OK;
}

ara_status ara_batch_autotune(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                              ara_portfolio *const *pfs, const ara_run_opts *opts,
                              void *const *d_ylt_layers, void *const *d_ylt_portfolio,
                              void *d_scratch, size_t scratch_bytes, void *stream,
                              ara_batch_config *best, double *best_ms) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!best) return fail(ctx, ARA_E_INVALID_ARG, "ara_batch_autotune: null result");
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    hipEvent_t e0, e1;
    ARA_HIP(ctx, hipEventCreate(&e0));
    ARA_HIP(ctx, hipEventCreate(&e1));
    const int tiles[] = {1, 2, 4};
    const int waves[] = {0, 16, 20};                   // 0: one workgroup per item
    const int orders[] = {ARA_BATCH_PORTFOLIO_MAJOR, ARA_BATCH_TRIAL_MAJOR};
    double bms = 1e300;
    ara_batch_config bc = {1, 0, ARA_BATCH_PORTFOLIO_MAJOR};
    ara_status st = ARA_OK;
    bool warm = false;
    for (int oi = 0; oi < 2 && st == ARA_OK; ++oi)
        for (int ti = 0; ti < 3 && st == ARA_OK; ++ti)
            for (int wi = 0; wi < 3 && st == ARA_OK; ++wi) {
                ara_batch_config c = {tiles[ti], waves[wi], orders[oi]};
                BatchPlan plan;
                st = prep_batch(ctx, yet, n_portfolios, pfs, opts, &c, d_ylt_layers,
                                d_ylt_portfolio, d_scratch, scratch_bytes, s, &plan);
                if (st != ARA_OK) break;
                hipError_t he = hipSuccess;
                if (!warm) {
                    he = launch_plan(ctx, yet, plan, s);
                    warm = true;
                }
                if (he == hipSuccess) he = hipEventRecord(e0, s);
                if (he == hipSuccess)
                    he = launch_plan(ctx, yet, plan, s);
                if (he == hipSuccess) he = hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                if (he != hipSuccess) {
                    st = fail(ctx, ARA_E_HIP, "ara_batch_autotune: %s", hipGetErrorString(he));
                    break;
                }
                if (ms < bms) {
                    bms = ms;
                    bc = c;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ARA_OK) return st;
    *best = bc;
    if (best_ms) *best_ms = bms;
    return check_status(ctx, s, "ara_batch_autotune");
}

ara_status ara_batch_graph_create(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                                  ara_portfolio *const *pfs, const ara_run_opts *opts,
                                  const ara_batch_config *cfg, void *const *d_ylt_layers,
                                  void *const *d_ylt_portfolio, void *d_scratch,
                                  size_t scratch_bytes, ara_graph **out) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!out) return fail(ctx, ARA_E_INVALID_ARG, "ara_batch_graph_create: null out");
    *out = nullptr;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t cap;
    ARA_HIP(ctx, hipStreamCreate(&cap));
    BatchPlan plan;
    // the portfolio table is copied eagerly; the graph holds only kernels
    ara_status st = prep_batch(ctx, yet, n_portfolios, pfs, opts, cfg, d_ylt_layers,
                               d_ylt_portfolio, d_scratch, scratch_bytes, cap, &plan);
    if (st == ARA_OK) {
        hipError_t he = hipStreamSynchronize(cap);
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        if (he == hipSuccess) he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
            hipError_t le = launch_plan(ctx, yet, plan, cap);
            he = hipStreamEndCapture(cap, &g);
            if (he == hipSuccess) he = le;
        }
        if (he == hipSuccess) he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (he != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            st = fail(ctx, ARA_E_HIP, "ara_batch_graph_create: %s", hipGetErrorString(he));
        } else {
            ara_graph *gr = new ara_graph();
            gr->graph = g;
            gr->exec = x;
            ctx->graphs.insert(gr);
            *out = gr;
        }
    }
    (void)hipStreamDestroy(cap);
    return st;
}

ara_status ara_graph_launch(ara_context *ctx, ara_graph *graph, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!graph || !ctx->graphs.count(graph))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_graph_launch: unknown graph");
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return ARA_OK;
}

ara_status ara_graph_destroy(ara_context *ctx, ara_graph *graph) {
    if (!ctx || !graph || !ctx->graphs.count(graph)) return ARA_E_INVALID_ARG;
    ctx->graphs.erase(graph);
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return ARA_OK;
}

ara_status ara_debug_philox(ara_context *ctx, int64_t n, const uint32_t *d_ctr, uint64_t key,
                            uint32_t *d_out, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!d_ctr || !d_out)))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_debug_philox: bad arguments");
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, launch_debug_philox(n, d_ctr, key, d_out, (hipStream_t)stream));
    return ARA_OK;
}

ara_status ara_debug_beta_quantile_shape(ara_context *ctx, int64_t n, float a, float b,
                                         const double *d_z, const double *d_zc, float *d_x,
                                         int32_t *d_path, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!d_z || !d_zc || !d_x)) ||
        !(a >= kF32MinShape && a <= kF32MaxShape) || !(b >= kF32MinShape && b <= kF32MaxShape))
        return fail(ctx, ARA_E_INVALID_ARG,
                    "ara_debug_beta_quantile_shape: bad arguments (a, b in [1, 32])");
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    void *mem = nullptr;
    float *tab = nullptr;
    ara_status st = one_shape_table(ctx, a, b, s, &mem, &tab);
    if (st != ARA_OK) {
        (void)hipFree(mem);
        return st;
    }
    // the per-entry shape arrays of the general diagnostic, all (a, b)
    void *ab = nullptr;
    hipError_t e = hipMalloc(&ab, sizeof(float) * 2 * (size_t)(n > 0 ? n : 1));
    if (e == hipSuccess && n > 0) {
        std::vector<float> h(2 * (size_t)n);
        for (int64_t j = 0; j < n; ++j) {
            h[(size_t)j] = a;
            h[(size_t)(n + j)] = b;
        }
        e = hipMemcpyAsync(ab, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_debug_quantile(n, (const float *)ab, (const float *)ab + n, d_z, d_zc,
                                      kDefaultTailBand, tab, d_x, d_path, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    (void)hipFree(ab);
    (void)hipFree(mem);
    if (e != hipSuccess)
        return fail(ctx, ARA_E_HIP, "ara_debug_beta_quantile_shape: %s", hipGetErrorString(e));
    return ARA_OK;
}

ara_status ara_debug_beta_quantile(ara_context *ctx, int64_t n, const float *d_a, const float *d_b,
                                   const double *d_z, const double *d_zc, float tail_band,
                                   float *d_x, int32_t *d_path, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!d_a || !d_b || !d_z || !d_zc || !d_x)))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_debug_beta_quantile: bad arguments");
    if (!(tail_band > 0.0f)) tail_band = kDefaultTailBand;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, launch_debug_quantile(n, d_a, d_b, d_z, d_zc, tail_band, nullptr, d_x, d_path,
                                       (hipStream_t)stream));
    return ARA_OK;
}

ara_status ara_probe_stream_read(ara_context *ctx, const void *d_src, size_t bytes,
                                 uint32_t *d_sink, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (!d_src || !d_sink || bytes % 16 != 0 || ((uintptr_t)d_src & 15) != 0)
        return fail(ctx, ARA_E_INVALID_ARG,
                    "ara_probe_stream_read: need a 16-byte aligned source and a multiple of 16 bytes");
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    ARA_HIP(ctx, launch_probe_stream(d_src, (int64_t)(bytes / 16), d_sink, ctx->n_cu,
                                     (hipStream_t)stream));
    return ARA_OK;
}

ara_status ara_probe_valu_lanes(ara_context *ctx, int32_t waves_per_simd, int64_t *lanes) {
    if (!ctx || !lanes || waves_per_simd < 1 || waves_per_simd > 8) return ARA_E_INVALID_ARG;
    *lanes = (int64_t)ctx->n_cu * waves_per_simd * 256;
    return ARA_OK;
}

ara_status ara_probe_valu(ara_context *ctx, int32_t kind, int32_t waves_per_simd, int32_t iters,
                          float *d_out, uint64_t *valu_instr, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (kind < ARA_PROBE_FMA_F32 || kind > ARA_PROBE_FMA_F64 || waves_per_simd < 1 ||
        waves_per_simd > 8 || iters < 1 || !d_out)
        return fail(ctx, ARA_E_INVALID_ARG, "ara_probe_valu: bad arguments");
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    // one 4-wavefront block per SIMD quadruple: waves_per_simd blocks per CU
    const int blocks = ctx->n_cu * waves_per_simd;
    ARA_HIP(ctx, launch_probe_valu(kind, blocks, iters, d_out, (hipStream_t)stream));
    // eight chains, one instruction per step (two for XAD and MAD_U64_U32)
    const uint64_t per_round =
        (kind == ARA_PROBE_XAD_U32 || kind == ARA_PROBE_MAD_U64_U32) ? 16u : 8u;
    if (valu_instr) *valu_instr = (uint64_t)blocks * 4u * per_round * (uint64_t)iters;
    return ARA_OK;
}

ara_status ara_probe_draws(ara_context *ctx, int64_t n, uint64_t seed, uint32_t elt_id, float a,
                           float b, int32_t use_shape_table, float *d_x, void *stream) {
    if (!ctx) return ARA_E_INVALID_ARG;
    if (n < 0 || (n > 0 && !d_x) || !(a >= kF32MinShape && a <= kF32MaxShape) ||
        !(b >= kF32MinShape && b <= kF32MaxShape))
        return fail(ctx, ARA_E_INVALID_ARG, "ara_probe_draws: bad arguments (a, b in [1, 32])");
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    // the row constants as the portfolio build makes them
    const double lnb = std::lgamma((double)a) + std::lgamma((double)b) -
                       std::lgamma((double)a + (double)b);
    const float lnb2 = (float)(lnb * 1.4426950408889634);
    int32_t h[2] = {0, 0};
    int32_t *d = (int32_t *)ctx->d_maxlen;     // 8 bytes of context scratch, free between loads
    ARA_HIP(ctx, launch_probe_row_consts(a, b, d, s));
    ARA_HIP(ctx, hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, s));
    ARA_HIP(ctx, hipStreamSynchronize(s));
    if (h[0] == 0 || h[1] == 0)
        return fail(ctx, ARA_E_UNSUPPORTED, "ara_probe_draws: shape needs the FP64 quantile");
    void *mem = nullptr;
    float *tab = nullptr;
    if (use_shape_table) {
        ara_status st = one_shape_table(ctx, a, b, s, &mem, &tab);
        if (st != ARA_OK) {
            (void)hipFree(mem);
            return st;
        }
    }
    hipError_t e = launch_probe_draws(n, seed, elt_id, a, b, lnb2, h[0], h[1], tab, d_x, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mem);
    if (e != hipSuccess) return fail(ctx, ARA_E_HIP, "ara_probe_draws: %s", hipGetErrorString(e));
    return ARA_OK;
}

}  // extern "C"

namespace ara {
ara_status run_batch_ranges(ara_context *ctx, const ara_yet *yet, int32_t n,
                            ara_portfolio *const *pfs, const ara_run_opts *opts,
                            const ara_batch_config *cfg, void *const *ylt_l, void *const *ylt_p,
                            const int64_t *ranges, void *scratch, size_t bytes, void *stream,
                            Status *status) {
    if (!ctx) return ARA_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    ARA_HIP(ctx, hipSetDevice(ctx->device));
    BatchPlan plan;
    ara_status st = prep_batch_ranges(ctx, yet, n, pfs, opts, cfg, ylt_l, ylt_p, ranges, scratch,
                                      bytes, s, status, &plan);
    if (st != ARA_OK) return st;
    ARA_HIP(ctx, launch_plan(ctx, yet, plan, s));
    return ARA_OK;
}
size_t batch_scratch_need(int32_t n, int64_t total_trials) { return batch_need(n, total_trials); }
}  // namespace ara

