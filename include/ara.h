/*
 * ara.h -- C-ABI of the MI355X (gfx950) Aggregate Risk Analysis library.
 *
 * Aggregate Risk Analysis (ARA) as defined in B. Varghese, "The GPU vs Phi
 * Debate: Risk Analytics Using Many-Core Computing": a Year Event Table (YET,
 * section 2.1 (i)) is run against a portfolio of layers, each covering a set
 * of Event Loss Tables (ELT / extended XELT, sections 2.1 (ii) and 3.1) under
 * occurrence and aggregate terms (section 2.1 (iii)); Algorithm 1 produces a
 * Year Loss Table (YLT, section 2.3) from which PML and TVaR are taken.
 * Secondary uncertainty (section 3) replaces each looked-up mean loss by a
 * Beta-distributed draw.
 *
 * Conventions for every entry point
 *  - Pointers named d_* are device pointers (memory of the context's GPU);
 *    all others are host pointers.  Streams are hipStream_t passed as void*
 *    (NULL = the null stream).
 *  - Every call returns an ara_status (0 = ARA_OK, negative on error) and
 *    never aborts; ara_last_error() gives a message for the last failure of
 *    a context.  A context is not thread-safe: use one per host thread.
 *  - Work is enqueued on the caller's stream; calls that return host values
 *    (ara_load_yet, ara_load_portfolio, ara_pml_tvar, ara_sync_status)
 *    synchronise that stream.
 *  - The library allocates no large device memory: the YET is borrowed from
 *    the caller, portfolio tables live in a caller-provided workspace, outputs
 *    and scratch are caller buffers.  A context keeps a few hundred bytes of
 *    device status words.
 *
 * Readings of points the paper leaves open (used identically by the tests'
 * FP64 reference):
 *  - ELT financial terms (section 2.2, Algorithm 1 "apply financial terms"):
 *    l' = share * min(max(loss - retention, 0), limit).
 *  - Occurrence terms on the event loss summed over a layer's ELTs; aggregate
 *    terms on the running sum of occurrence losses (section 2.2), never fed
 *    back into that sum.  The trial loss is the aggregate value after the
 *    last occurrence.  Because occurrence losses are >= 0 and the aggregate
 *    clamp is monotone, that value equals the clamp of the total, so the
 *    device may sum a trial's occurrences in any order.
 *  - Secondary uncertainty draws: Philox4x32-10 (Salmon et al., SC'11),
 *    counter (k, i, elt_id, 0) for the independent uniform and (k, i, 0, 1)
 *    for the correlated one, key (seed low 32 bits, seed high 32 bits), output
 *    word 0 mapped to u = ((w >> 8) | 1) * 2^-24.  k = occurrence index in
 *    the trial, i = absolute trial index.  sigma_C = 0 gives z = u_I and
 *    sigma_I = 0 gives z = u_C exactly (section 3.2's extreme cases).
 *  - Beta fit (section 3.3) with sigma = sigma_I + sigma_C; when
 *    sigma/max_l >= sqrt(mu_b (1 - mu_b)) the cap uses (1 - 1e-6) times it.
 *  - PML(RP) = k-th largest trial loss, TVaR(RP) = mean of the k largest,
 *    k = max(1, floor(N / RP)).
 */
#ifndef ARA_H
#define ARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ara_status;

enum {
    ARA_OK = 0,
    ARA_E_INVALID_ARG = -1,          /* a null/negative/inconsistent argument */
    ARA_E_NO_DEVICE = -2,            /* the HIP device does not exist */
    ARA_E_HIP = -3,                  /* a HIP runtime call failed (message has it) */
    ARA_E_EVENT_ID_RANGE = -4,       /* an event id outside [0, n_catalogue) */
    ARA_E_OFFSETS_NOT_MONOTONE = -5, /* YET trial offsets decrease or do not start at 0 */
    ARA_E_TIMES_UNSORTED = -6,       /* time stamps decrease inside a trial */
    ARA_E_BAD_ELT_ROW = -7,          /* NaN/negative value, mean >= max_loss with sigma > 0,
                                        duplicate event in one ELT, share outside [0, 1],
                                        negative retention */
    ARA_E_WORKSPACE_TOO_SMALL = -8,  /* workspace / scratch smaller than required */
    ARA_E_NUMERIC = -9,              /* a Beta quantile failed to converge */
    ARA_E_UNSUPPORTED = -10          /* option combination not supported */
};

/* How a trial's occurrence losses are summed: compensated FP32 (Neumaier;
 * the default, value 0), plain FP32, or FP64. */
enum { ARA_SUM_KAHAN32 = 0, ARA_SUM_NAIVE32 = 1, ARA_SUM_F64 = 2 };
enum { ARA_F32 = 0, ARA_F64 = 1 };

typedef struct ara_context ara_context;
typedef struct ara_yet ara_yet;
typedef struct ara_portfolio ara_portfolio;

/* One ELT / XELT (sections 2.1 (ii), 3.1).  Host arrays of n_rows entries,
 * copied during ara_load_portfolio.  sigma_i, sigma_c and max_loss may be
 * NULL (all zero; then the ELT has no secondary uncertainty). */
typedef struct {
    uint32_t elt_id;            /* caller's id; keys the random draws */
    int32_t n_rows;
    const int32_t *event_ids;   /* distinct, in [0, n_catalogue) */
    const float *mean;          /* mean loss mu_l >= 0 */
    const float *sigma_i;       /* independent standard deviation */
    const float *sigma_c;       /* correlated standard deviation */
    const float *max_loss;      /* exposure max_l > mean where sigma > 0 */
    double retention, limit, share;   /* ELT financial terms (limit may be +inf) */
} ara_elt_desc;

/* One layer: its ELTs (in order) and the layer terms (section 2.1 (iii)). */
typedef struct {
    int32_t n_elts;
    const ara_elt_desc *elts;
    double occ_retention, occ_limit, agg_retention, agg_limit;   /* limits may be +inf */
    uint32_t program_id;        /* label only */
} ara_layer_desc;

/* How the two uniforms of section 3.2 are keyed (Philox4x32-10 counter words
 * (c0, c1, c2, c3), key = the portfolio seed; k = occurrence index in the
 * trial, i = absolute trial index, E = event id):
 *   ARA_KEYING_OCCURRENCE (default): u_I at (k, i, elt_id, 0), independent
 *     per ELT; u_C at (k, i, 0, 1), shared by every ELT of the occurrence.
 *   ARA_KEYING_PAPER (the inputs of section 3.1 as laid out there): u_I is
 *     z_(Prog,E), one per occurrence and program, at (k, i, program_id, 2),
 *     shared by all ELTs of the program's layers; u_C is z_(E), the value an
 *     XELT row holds for its event, the same in every occurrence, ELT and
 *     program, at (E, 0, 0, 3). */
#define ARA_KEYING_OCCURRENCE 0
#define ARA_KEYING_PAPER 1

typedef struct {
    int32_t n_layers;
    const ara_layer_desc *layers;
    uint64_t seed;              /* Philox key */
    int32_t su_enabled;         /* 0: primary uncertainty only (mean losses) */
    int32_t keying;             /* ARA_KEYING_* */
} ara_portfolio_desc;

typedef struct {
    int64_t trial_begin;        /* first absolute trial of the run */
    int64_t trial_count;        /* number of trials; -1 = to the end of the YET */
    int32_t sum_mode;           /* ARA_SUM_*: how a trial's occurrence losses are summed */
    int32_t ylt_dtype;          /* ARA_F32 or ARA_F64 for both YLT outputs */
    float tail_band;            /* z or 1-z below this use the FP64 quantile; <= 0: 2^-24 */
    int32_t debug_flags;        /* 0, or ARA_DEBUG_* (tests of the failure paths) */
    int64_t *d_hits;            /* optional [n_layers][trial_count]: non-zero lookups */
    uint64_t *d_hit_chk;        /* optional [n_layers][trial_count]: sum over hits of
                                   (k+1)*2654435761 + elt_id, modulo 2^64 */
    void *d_scratch;            /* ara_run_scratch_size(trial_count) bytes of device scratch
                                   (the trials handed from the FP32 pass to the FP64-capable
                                   pass); required for portfolios with secondary
                                   uncertainty, unused without.  Runs that overlap in time
                                   need scratch of their own. */
    size_t scratch_bytes;
    void *d_occ_view;           /* optional occurrence view (section 2.2, aggregate terms):
                                   element l * occ_view_stride + (j - offsets[trial_begin])
                                   receives, for occurrence j of the run's trials, layer l's
                                   increment d_j = A_j - A_{j-1} of the aggregate-term output
                                   A_j = min(max(S_j - AggR, 0), AggL) over the running sum
                                   S_j of the trial's occurrence losses in stored (time)
                                   order; S_j in FP64; elements in opts->ylt_dtype.  A trial's
                                   increments add up to its layer loss (up to rounding). */
    int64_t occ_view_stride;    /* elements per layer of d_occ_view (>= the run's
                                   occurrences; a larger index is not written and the run
                                   reports ARA_E_WORKSPACE_TOO_SMALL through ara_sync_status) */
} ara_run_opts;

/* ara_run_opts.debug_flags.  ARA_DEBUG_QUANTILE_ONE_STEP sends every draw to
 * the FP64 quantile and lets that iteration take a single step, so draws
 * whose start is not already a root are reported as non-converging
 * (ARA_E_NUMERIC through ara_sync_status) while every kernel ends normally;
 * for tests of the convergence check (section 5.1's criterion) only. */
#define ARA_DEBUG_QUANTILE_ONE_STEP 1

/* ---- context ------------------------------------------------------------ */
ara_status ara_create(int hip_device, ara_context **out);
void ara_destroy(ara_context *ctx);               /* frees outstanding handles too */
const char *ara_status_string(ara_status s);
const char *ara_last_error(const ara_context *ctx);

/* ---- Year Event Table (section 2.1 (i)) ---------------------------------
 * CSR by trial: trial t holds occurrences [d_trial_offsets[t],
 * d_trial_offsets[t+1]) of d_event_ids (int32, 0-based catalogue ids; may be
 * NULL when d_trial_offsets[n_trials] == 0, a YET of empty trials) and
 * d_times (float32 time stamps, may be NULL).  The arrays are borrowed and
 * must stay alive and unchanged until ara_free_yet.  Validates on the device
 * (ids in range, offsets[0] == 0 and non-decreasing, times non-decreasing
 * inside each trial) and synchronises the stream. */
ara_status ara_load_yet(ara_context *ctx, int64_t n_trials, int32_t n_catalogue,
                        const int64_t *d_trial_offsets, const int32_t *d_event_ids,
                        const float *d_times, void *stream, ara_yet **out);
ara_status ara_free_yet(ara_context *ctx, ara_yet *yet);

/* ---- portfolio (sections 2.1 (iii), 3.1, 3.3, 4.2) -----------------------
 * ara_portfolio_workspace_size gives the bytes of device workspace that
 * ara_load_portfolio needs for this description and catalogue size.
 * ara_load_portfolio validates the rows, copies them into d_workspace and
 * builds there, with device kernels, each layer's event-indexed direct-access
 * structure and the per-row Beta fit; it synchronises the stream.  The
 * workspace belongs to the portfolio until ara_free_portfolio; the host
 * arrays of the description may be freed on return.  Both return
 * ARA_E_UNSUPPORTED for a layer of 2^27 or more ELT rows (the compact row
 * records hold a layer-local row index in 27 bits) or a portfolio of 2^32 or
 * more. */
ara_status ara_portfolio_workspace_size(const ara_portfolio_desc *desc, int32_t n_catalogue,
                                        size_t *bytes);
ara_status ara_load_portfolio(ara_context *ctx, const ara_portfolio_desc *desc,
                              int32_t n_catalogue, void *d_workspace, size_t bytes,
                              void *stream, ara_portfolio **out);
ara_status ara_free_portfolio(ara_context *ctx, ara_portfolio *pf);

/* ---- the analysis (Algorithm 1 with secondary uncertainty) ---------------
 * Runs trials [trial_begin, trial_begin + trial_count) and writes
 * d_ylt_layers[l * trial_count + t] (loss of layer l in trial trial_begin+t)
 * and d_ylt_portfolio[t] (sum over layers), in opts->ylt_dtype; either output
 * may be NULL.  opts may be NULL (all trials, KAHAN32, F32) for portfolios
 * without secondary uncertainty; with it, opts->d_scratch is required
 * (ARA_E_WORKSPACE_TOO_SMALL otherwise).  The call allocates nothing.
 * Asynchronous: returns after enqueueing on the stream; a quantile failure is
 * reported by ara_sync_status. */
ara_status ara_run(ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                   const ara_run_opts *opts, void *d_ylt_layers, void *d_ylt_portfolio,
                   void *stream);

/* Device scratch an ara_run over trial_count trials needs (the list of
 * trials handed from the FP32 pass to the FP64-capable pass). */
ara_status ara_run_scratch_size(int64_t trial_count, size_t *bytes);

/* ara_run for callers that cannot allocate device memory at all (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc): the
 * same run and the same results as ara_run, but the hand-over scratch is a
 * device array the library holds on every GPU it runs on, for the life of
 * the process (ARA_STATIC_MAX_TRIALS x 4 + 256 bytes, 16 MiB), so
 * opts->d_scratch is ignored and the call allocates nothing; the caller still
 * passes the inputs and outputs.  A run of more than ARA_STATIC_MAX_TRIALS
 * trials fails with ARA_E_WORKSPACE_TOO_SMALL.  Every call on one GPU
 * shares that array (the counter is cleared by a kernel at the start of each
 * call): calls that overlap in time on one GPU -- on two streams, or from two
 * contexts of the same device -- race and must be serialised by the caller.
 * Asynchronous, as ara_run. */
#define ARA_STATIC_MAX_TRIALS (1 << 22)
ara_status ara_run_static(ara_context *ctx, const ara_yet *yet, const ara_portfolio *pf,
                          const ara_run_opts *opts, void *d_ylt_layers, void *d_ylt_portfolio,
                          void *stream);

/* Synchronises the stream and reports ARA_E_NUMERIC (with the first failing
 * trial, occurrence and elt_id in the message) if a run since the last call
 * hit a non-converging quantile; clears the flag. */
ara_status ara_sync_status(ara_context *ctx, void *stream);

/* ---- batched portfolios --------------------------------------------------
 * Several portfolios (Algorithm 1's outer portfolio / program loops) over one
 * YET in one persistent launch.  Work items are (tile of trial_tile trials,
 * portfolio), handed out from an atomic counter in one of two orders:
 * portfolio-major (each portfolio's tiles in turn: its ELT tables stay in the
 * caches, the better order when the draws dominate) or trial-major (the
 * portfolios of one tile together: the tile's event ids are read once for all
 * of them, the better order for primary-uncertainty batches, which are bound
 * by memory traffic).  Results are bit-identical to running each portfolio
 * alone with ara_run: the secondary-uncertainty portfolios share the one
 * launch, and each primary-uncertainty portfolio runs ara_run's per-event
 * table pass after it on the same stream (captured with it by
 * ara_batch_graph_create).  d_ylt_layers /
 * d_ylt_portfolio are host arrays of n_portfolios device pointers (entries
 * may be NULL), laid out as for ara_run over opts->trial_count trials.
 * opts->d_hits / d_hit_chk must be NULL; its d_scratch is not used (the batch
 * scratch is the explicit argument, ara_batch_scratch_size bytes).
 * The launch takes one of two forms: one workgroup per work item (the
 * hardware dispatcher hands items out in order as wavefronts retire), or a
 * persistent grid of waves_per_cu wavefronts per CU that take items from an
 * atomic counter.  cfg = NULL: trial_tile 1, one workgroup per item,
 * portfolio-major unless every portfolio is primary-uncertainty. */
#define ARA_BATCH_PORTFOLIO_MAJOR 0
#define ARA_BATCH_TRIAL_MAJOR 1
typedef struct {
    int32_t trial_tile;         /* trials per work item (>= 1) */
    int32_t waves_per_cu;       /* 0: one workgroup per work item (at most 2^31 - 1 items);
                                   > 0: persistent form, resident wavefronts per CU */
    int32_t order;              /* ARA_BATCH_PORTFOLIO_MAJOR or ARA_BATCH_TRIAL_MAJOR */
} ara_batch_config;

ara_status ara_batch_scratch_size(int32_t n_portfolios, int64_t trial_count, size_t *bytes);
ara_status ara_run_batch(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                         ara_portfolio *const *pfs, const ara_run_opts *opts,
                         const ara_batch_config *cfg, void *const *d_ylt_layers,
                         void *const *d_ylt_portfolio, void *d_scratch, size_t scratch_bytes,
                         void *stream);

/* Autotuner: times ara_run_batch over opts' trial range (HIP events, after
 * one warmup launch) for trial tiles {1, 2, 4} x waves per CU {0 (one
 * workgroup per item), 16, 20} x both orders and returns the fastest
 * configuration and its time.  A range of a few thousand trials keeps it to
 * seconds.  Synchronises. */
ara_status ara_batch_autotune(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                              ara_portfolio *const *pfs, const ara_run_opts *opts,
                              void *const *d_ylt_layers, void *const *d_ylt_portfolio,
                              void *d_scratch, size_t scratch_bytes, void *stream,
                              ara_batch_config *best, double *best_ms);

/* The same batched run captured once in a HIP graph (no host work between
 * replays); the graph keeps the pointers it was built with, which must stay
 * valid while it exists.  ara_graph_launch replays it on the stream. */
typedef struct ara_graph ara_graph;
ara_status ara_batch_graph_create(ara_context *ctx, const ara_yet *yet, int32_t n_portfolios,
                                  ara_portfolio *const *pfs, const ara_run_opts *opts,
                                  const ara_batch_config *cfg, void *const *d_ylt_layers,
                                  void *const *d_ylt_portfolio, void *d_scratch,
                                  size_t scratch_bytes, ara_graph **out);
ara_status ara_graph_launch(ara_context *ctx, ara_graph *graph, void *stream);
ara_status ara_graph_destroy(ara_context *ctx, ara_graph *graph);

/* ---- serving ------------------------------------------------------------
 * A request loop over a YET resident in HBM.  Portfolio-pricing requests
 * (a portfolio description, a trial range, return periods) are queued by
 * ara_server_submit from any host thread; a worker thread admits them in
 * arrival order as far as their HBM footprint (portfolio workspace, YLT
 * outputs, metric scratch) fits the caller's device pool, launches every
 * admitted group as one batched launch with a trial range per request on one
 * of max_inflight streams -- so groups admitted while others run overlap on
 * the device -- and on completion takes PML / TVaR and records latencies.
 * A request's result does not depend on what it was batched with: it is bit
 * for bit the result of the same request submitted alone (the draws are keyed
 * by trial, occurrence and ELT id, and each trial is summed by one wavefront).
 * It also equals ara_run over the same trials bit for bit (primary-
 * uncertainty portfolios run ara_run's per-event table pass).  The server
 * creates one context per stream on
 * hip_device; the YET arrays and the pool are borrowed and must outlive the
 * server.  A request that fails validation fails alone (its result carries
 * the status; ara_server_last_error gives the message of the last failure). */
typedef struct ara_server ara_server;

typedef struct {
    int32_t max_inflight;       /* request groups in flight (streams); <= 0: 4 */
    int32_t max_batch;          /* requests per batched launch; <= 0: 16 */
    int32_t sum_mode;           /* ARA_SUM_* (0: KAHAN32) */
    int32_t reserved;
    void *d_pool;               /* device memory the server sub-allocates requests from */
    size_t pool_bytes;
} ara_server_config;

#define ARA_SERVER_MAX_RP 16

typedef struct {
    uint64_t request_id;
    ara_status status;
    int32_t n_rp;
    double pml[ARA_SERVER_MAX_RP];
    double tvar[ARA_SERVER_MAX_RP];
    double queue_s;             /* submission -> launch of its group */
    double latency_s;           /* submission -> PML / TVaR ready on the host */
    const float *ylt;           /* host copy of the portfolio YLT if requested, else NULL;
                                   valid until ara_server_release(request_id) */
    int64_t ylt_count;
} ara_server_result;

ara_status ara_server_create(int hip_device, int64_t n_trials, int32_t n_catalogue,
                             const int64_t *d_trial_offsets, const int32_t *d_event_ids,
                             const ara_server_config *cfg, ara_server **out);
/* flags: ARA_SUBMIT_WANT_YLT returns a host copy of the portfolio YLT with
 * the result; ARA_SUBMIT_BORROW keeps pointers to the description's row
 * arrays instead of copying them (the caller keeps them valid and unchanged
 * until the request's result has been polled); without it the description is
 * copied during the call.  Fails with ARA_E_WORKSPACE_TOO_SMALL when the
 * request alone can never fit the pool. */
#define ARA_SUBMIT_WANT_YLT 1
#define ARA_SUBMIT_BORROW 2
ara_status ara_server_submit(ara_server *srv, const ara_portfolio_desc *desc, int64_t trial_begin,
                             int64_t trial_count, const double *return_periods, int32_t n_rp,
                             int32_t flags, uint64_t *request_id);
/* Up to max_results finished requests (waiting up to wait_s seconds for the
 * first one); *n_out receives the count. */
ara_status ara_server_poll(ara_server *srv, ara_server_result *out, int32_t max_results,
                           double wait_s, int32_t *n_out);
ara_status ara_server_release(ara_server *srv, uint64_t request_id);
/* Stops after the queued and running requests finish, joins the worker. */
ara_status ara_server_destroy(ara_server *srv);
/* Message of the most recent failed request; the pointer stays valid in the
 * calling thread until its next call. */
const char *ara_server_last_error(ara_server *srv);

/* ---- risk metrics (section 2.3) -------------------------------------------
 * PML and TVaR of the n losses in d_ylt (ARA_F32 or ARA_F64, all >= 0) for
 * n_rp return periods; results to host arrays pml_out / tvar_out.  The k-th
 * largest value is found by a device radix select over the bit patterns; the
 * tail sum is accumulated in FP64.  d_scratch must hold
 * ara_pml_tvar_scratch_size(n) bytes.  Synchronises the stream. */
ara_status ara_pml_tvar_scratch_size(int64_t n, size_t *bytes);
ara_status ara_pml_tvar(ara_context *ctx, const void *d_ylt, int32_t ylt_dtype, int64_t n,
                        const double *return_periods, int32_t n_rp, double *pml_out,
                        double *tvar_out, void *d_scratch, size_t scratch_bytes, void *stream);

/* Exceedance-probability curve (the return-period losses of section 2.3's
 * reports) of the n losses in d_ylt (all >= 0): d_sorted[j] (n elements of
 * ylt_dtype) receives the losses in descending order, so d_sorted[j] is the
 * loss exceeded or equalled in a fraction (j+1)/n of the trials (return
 * period n/(j+1)); d_tail_mean[j] (n doubles, may be NULL) the FP64 mean of
 * d_sorted[0..j], the TVaR at that point.  For a return period RP with
 * k = max(1, floor(n/RP)), d_sorted[k-1] and d_tail_mean[k-1] are the PML and
 * TVaR of ara_pml_tvar.  -0.0 sorts as +0.0.  d_sorted may not alias d_ylt.
 * d_scratch must hold ara_ep_curve_scratch_size(n, ylt_dtype) bytes.
 * Asynchronous: enqueued on the stream. */
ara_status ara_ep_curve_scratch_size(int64_t n, int32_t ylt_dtype, size_t *bytes);
ara_status ara_ep_curve(ara_context *ctx, const void *d_ylt, int32_t ylt_dtype, int64_t n,
                        void *d_sorted, double *d_tail_mean, void *d_scratch,
                        size_t scratch_bytes, void *stream);

/* ---- diagnostics (used by the tests) -------------------------------------
 * ara_debug_philox: d_out[4j..4j+3] = Philox4x32-10(d_ctr[4j..4j+3], key).
 * ara_debug_beta_quantile: d_x[j] = I^-1(z_j; a_j, b_j) by the same device
 * code the analysis uses (FP32, FP64 below tail_band (<= 0: 2^-24) and for
 * shapes the FP32 path does not cover), given z and its complement zc = 1 - z (FP64
 * inputs, exact grid values) and a per-entry FP32 shape; d_path[j] (may be
 * NULL) receives 0 for the FP32 path, 1 for the FP64 path. */
ara_status ara_debug_philox(ara_context *ctx, int64_t n, const uint32_t *d_ctr, uint64_t key,
                            uint32_t *d_out, void *stream);
ara_status ara_debug_beta_quantile(ara_context *ctx, int64_t n, const float *d_a,
                                   const float *d_b, const double *d_z, const double *d_zc,
                                   float tail_band, float *d_x, int32_t *d_path, void *stream);
/* ara_debug_beta_quantile_shape: the same for n draws of one shape (a, b in
 * [1, 32]) through the path of rows whose shape has a table: the table is
 * built as a portfolio load builds it (in device memory allocated for the
 * call) and the FP32 quantile starts from it.  Synchronises the stream. */
ara_status ara_debug_beta_quantile_shape(ara_context *ctx, int64_t n, float a, float b,
                                         const double *d_z, const double *d_zc, float *d_x,
                                         int32_t *d_path, void *stream);

/* ---- measurement probes (the roofline figures of the benchmark) -----------
 * ara_probe_stream_read: reads bytes (a multiple of 16) of device memory at
 *   d_src (16-byte aligned) once with 16-byte non-temporal loads, the access
 *   pattern of the event-id stream, and XORs a digest into *d_sink (one
 *   device word); the duration gives the streaming bandwidth of the part.
 *   Asynchronous.
 * ara_probe_valu: eight independent chains of one vector instruction kind per
 *   lane (ARA_PROBE_*), iters rounds, waves_per_simd wavefronts on each SIMD of
 *   the device; d_out receives one float per lane (n_cu * 4 * waves_per_simd *
 *   64 floats, ara_probe_valu_lanes) and *valu_instr (host) the wavefront
 *   instructions of the chains (8 * iters per wavefront; 16 * iters for
 *   ARA_PROBE_XAD_U32, an xor and an add, and ARA_PROBE_MAD_U64_U32, a
 *   product and an xor).  Asynchronous.
 * ara_probe_draws: the per-draw arithmetic of secondary uncertainty alone
 *   (section 3): n draws of one ELT row of shape (a, b), Philox4x32-10 keyed
 *   (j mod 1024, j / 1024, elt_id, 0) with key = seed, the draw on the 2^-24
 *   grid and the FP32 Beta quantile (the analysis' bulk path), started from
 *   the shape's table when use_shape_table is non-zero (the path of rows
 *   whose shape has a table) or from the closed-form guess otherwise; d_x[j]
 *   receives the quantile (-1 where the FP32 iteration did not converge).
 *   a, b must lie in [1, 32].  Synchronises the stream (the quantile's
 *   continued-fraction term counts and the table are made on the device
 *   first, the table in 1.3 KB of device memory allocated for the call). */
enum {
    ARA_PROBE_FMA_F32 = 0,     /* v_fma_f32 */
    ARA_PROBE_MUL_F32 = 1,     /* v_mul_f32 */
    ARA_PROBE_XAD_U32 = 2,     /* (x ^ m) + c */
    ARA_PROBE_MULHI_U32 = 3,   /* high word of a 32 x 32 product (Philox) */
    ARA_PROBE_MAD_U64_U32 = 4, /* full 64-bit 32 x 32 product, halves xor-ed (Philox) */
    ARA_PROBE_EXP2_F32 = 5,    /* transcendental 2^x */
    ARA_PROBE_FMA_F64 = 6      /* v_fma_f64 */
};
ara_status ara_probe_stream_read(ara_context *ctx, const void *d_src, size_t bytes,
                                 uint32_t *d_sink, void *stream);
ara_status ara_probe_valu_lanes(ara_context *ctx, int32_t waves_per_simd, int64_t *lanes);
ara_status ara_probe_valu(ara_context *ctx, int32_t kind, int32_t waves_per_simd, int32_t iters,
                          float *d_out, uint64_t *valu_instr, void *stream);
ara_status ara_probe_draws(ara_context *ctx, int64_t n, uint64_t seed, uint32_t elt_id, float a,
                           float b, int32_t use_shape_table, float *d_x, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ARA_H */
