// ara_serve.hip -- serving loop: a YET resident in HBM; portfolio-pricing
// requests admitted by HBM footprint, their tables built ahead of time, and
// run in batched launches that queue back to back on the device (continuous
// batching); PML / TVaR are computed on the device behind each launch and
// reach the host with the completion event.
//
// One worker thread drives three stages, each pass in this order:
//   completions  a launch whose event has fired: read its results from pinned
//                memory, free the requests' pool regions;
//   launches     a free slot takes up to max_batch loaded requests (arrival
//                order) into one batched launch on its stream, followed by
//                each request's PML / TVaR and the copies of the results;
//   loads        the oldest submitted request is given a pool region and its
//                portfolio tables are built and validated on the load stream,
//                while the launches already queued keep the device busy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ara.h"
#include "ara_internal.h"
#include "ara_kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t) {
    return std::chrono::duration<double>(t - t0).count();
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over the caller's device pool (offsets only).
class PoolAllocator {
  public:
    explicit PoolAllocator(size_t bytes) { free_[0] = bytes; }
    bool alloc(size_t n, size_t *off) {
        n = align_up(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n ? n : 1);
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, sorted
};

// A request with its own copy of the portfolio description.  Its pool region
// holds, in order: portfolio workspace, layer YLT, portfolio YLT, PML / TVaR
// scratch, and the 2 x n_rp device results.
struct Request {
    uint64_t id = 0;
    std::vector<std::vector<int32_t>> ev;
    std::vector<std::vector<float>> mean, si, sc, mx;
    std::vector<std::vector<ara_elt_desc>> elts;
    std::vector<ara_layer_desc> layers;
    ara_portfolio_desc desc{};
    int64_t trial_begin = 0, trial_count = 0;
    std::vector<double> rps;
    std::vector<int64_t> ks;
    int want_ylt = 0;
    size_t ws_bytes = 0, ylt_l_bytes = 0, ylt_p_bytes = 0, pml_bytes = 0, out_bytes = 0;
    size_t footprint = 0;
    size_t off = 0;                    // pool offset of the region
    ara_portfolio *pf = nullptr;
    Clock::time_point t_submit, t_launch, t_done;
    ara_server_result res{};
    std::vector<float> ylt_host;
};

// Pinned host block of one slot: the launch's device status, then 2 x
// ARA_SERVER_MAX_RP doubles per request of the group.
struct HostBlock {
    ara::Status status;
    double out[1];
};

// One stream of the continuous batch, with its own device status word and
// batch scratch (sized for max_batch requests covering n_trials trials).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ara::Status *d_status = nullptr;
    HostBlock *h = nullptr;
    size_t scratch_off = 0, scratch_bytes = 0;
    bool busy = false;
    std::vector<Request *> reqs;
};

}  // namespace

struct ara_server {
    int device = 0;
    ara_context *ctx = nullptr;          // loads, runs and metrics (worker thread only)
    ara_yet *yet = nullptr;
    hipStream_t load_stream = nullptr;
    ara_server_config cfg{};
    char *pool = nullptr;
    PoolAllocator *alloc = nullptr;      // guarded by mu
    int32_t n_catalogue = 0;
    int64_t n_trials = 0;
    size_t request_room = 0;             // pool bytes left for requests
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;       // submitted (guarded by mu)
    std::deque<Request *> ready;         // loaded, not launched (worker only)
    std::deque<Request *> finished;      // guarded by mu
    std::map<uint64_t, Request *> handed_out;   // polled, not yet released (guarded by mu)
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    std::string err;

    void run();
    bool complete(Slot &s);
    bool launch(Slot &s);
    bool load_one();
    void finish(Request *r, ara_status st);
    void set_error(const Request *r);
    void destroy_all();
};

namespace {

ara_status request_footprint(ara_server *srv, Request *r) {
    size_t ws = 0;
    ara_status st = ara_portfolio_workspace_size(&r->desc, srv->n_catalogue, &ws);
    if (st != ARA_OK) return st;
    r->ws_bytes = align_up(ws);
    r->ylt_l_bytes = align_up(sizeof(float) * (size_t)r->desc.n_layers * (size_t)r->trial_count);
    r->ylt_p_bytes = align_up(sizeof(float) * (size_t)r->trial_count);
    r->pml_bytes = align_up(ara::pml_scratch_bytes(r->trial_count));
    r->out_bytes = align_up(sizeof(double) * 2 * ARA_SERVER_MAX_RP);
    r->footprint = r->ws_bytes + r->ylt_l_bytes + r->ylt_p_bytes + r->pml_bytes + r->out_bytes;
    return ARA_OK;
}

// k-th largest index of each return period: k = max(1, floor(N / RP)).
void metric_ranks(Request *r) {
    r->ks.resize(r->rps.size());
    for (size_t i = 0; i < r->rps.size(); ++i) {
        const double kk = std::floor((double)r->trial_count / r->rps[i]);
        r->ks[i] = kk < 1.0 ? 1 : (kk > (double)r->trial_count ? r->trial_count : (int64_t)kk);
    }
}

size_t slot_scratch_bytes(int32_t max_batch, int64_t n_trials) {
    return align_up(ara::batch_scratch_need(max_batch, n_trials));
}

}  // namespace

void ara_server::set_error(const Request *r) {
    std::lock_guard<std::mutex> lk(mu);
    err = "request " + std::to_string(r->id) + ": " + ara_last_error(ctx);
}

// Stamps a request's result and hands it to ara_server_poll.
void ara_server::finish(Request *r, ara_status st) {
    r->res.status = st;
    if (r->pf) ara_free_portfolio(ctx, r->pf);
    r->pf = nullptr;
    r->t_done = Clock::now();
    if (r->t_launch == Clock::time_point()) r->t_launch = r->t_done;
    r->res.request_id = r->id;
    r->res.n_rp = (int32_t)r->rps.size();
    r->res.queue_s = seconds_since(r->t_submit, r->t_launch);
    r->res.latency_s = seconds_since(r->t_submit, r->t_done);
    std::lock_guard<std::mutex> lk(mu);
    alloc->release(r->off, r->footprint);
    finished.push_back(r);
    cv_done.notify_all();
}

// Loads the oldest submitted request if its region fits the pool (a request
// that does not fit holds back those behind it: arrival order is kept).
bool ara_server::load_one() {
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (pending.empty()) return false;
        size_t off;
        if (!alloc->alloc(pending.front()->footprint, &off)) return false;
        r = pending.front();
        pending.pop_front();
        r->off = off;
    }
    ara_status st = ara_load_portfolio(ctx, &r->desc, n_catalogue, pool + r->off, r->ws_bytes,
                                       load_stream, &r->pf);
    if (st != ARA_OK) {
        r->pf = nullptr;
        set_error(r);
        finish(r, st);               // a request that fails validation fails alone
        return true;
    }
    ready.push_back(r);
    return true;
}

// Enqueues one batched launch of the oldest loaded requests on the slot's
// stream, then per request its PML / TVaR and the copy of the results, then
// the copy of the launch's status and the completion event.
bool ara_server::launch(Slot &s) {
    if (ready.empty()) return false;
    std::vector<Request *> group;
    int64_t total = 0;
    while (!ready.empty() && (int)group.size() < cfg.max_batch &&
           total + ready.front()->trial_count <= n_trials) {
        total += ready.front()->trial_count;
        group.push_back(ready.front());
        ready.pop_front();
    }
    std::vector<ara_portfolio *> pfs;
    std::vector<void *> yl, yp;
    std::vector<int64_t> ranges;
    const Clock::time_point now = Clock::now();
    for (Request *r : group) {
        char *base = pool + r->off;
        r->t_launch = now;
        pfs.push_back(r->pf);
        yl.push_back(base + r->ws_bytes);
        yp.push_back(base + r->ws_bytes + r->ylt_l_bytes);
        ranges.push_back(r->trial_begin);
        ranges.push_back(r->trial_count);
    }
    ara_run_opts o;
    std::memset(&o, 0, sizeof o);
    o.sum_mode = cfg.sum_mode;
    o.ylt_dtype = ARA_F32;
    // one trial per work item, one workgroup per item: small requests still
    // fill the chip, at the single-portfolio kernel's occupancy
    const ara_batch_config bc = {1, 0, ARA_BATCH_PORTFOLIO_MAJOR};
    ara_status st = ARA_OK;
    if (hipMemsetAsync(s.d_status, 0, sizeof(ara::Status), s.stream) != hipSuccess) st = ARA_E_HIP;
    if (st == ARA_OK)
        st = ara::run_batch_ranges(ctx, yet, (int32_t)pfs.size(), pfs.data(), &o, &bc, yl.data(),
                                   yp.data(), ranges.data(), pool + s.scratch_off,
                                   s.scratch_bytes, s.stream, s.d_status);
    for (size_t i = 0; i < group.size() && st == ARA_OK; ++i) {
        Request *r = group[i];
        char *pml = (char *)yp[i] + r->ylt_p_bytes;
        double *d_out = (double *)(pml + r->pml_bytes);
        if (ara::launch_pml_tvar(yp[i], ARA_F32, r->trial_count, r->ks.data(),
                                 (int32_t)r->ks.size(), pml, d_out, s.stream) != hipSuccess ||
            hipMemcpyAsync(s.h->out + i * 2 * ARA_SERVER_MAX_RP, d_out,
                           sizeof(double) * 2 * r->ks.size(), hipMemcpyDeviceToHost,
                           s.stream) != hipSuccess)
            st = ARA_E_HIP;
    }
    if (st == ARA_OK &&
        (hipMemcpyAsync(&s.h->status, s.d_status, sizeof(ara::Status), hipMemcpyDeviceToHost,
                        s.stream) != hipSuccess ||
         hipEventRecord(s.done, s.stream) != hipSuccess))
        st = ARA_E_HIP;
    if (st != ARA_OK) {
        // nothing of the group is left in flight once the stream has drained
        (void)hipStreamSynchronize(s.stream);
        for (Request *r : group) {
            set_error(r);
            finish(r, st);
        }
        return true;
    }
    s.reqs = group;
    s.busy = true;
    return true;
}

bool ara_server::complete(Slot &s) {
    if (!s.busy || hipEventQuery(s.done) != hipSuccess) return false;
    ara_status group_st = s.h->status.code == 0 ? ARA_OK : (ara_status)s.h->status.code;
    if (group_st != ARA_OK) {
        std::lock_guard<std::mutex> lk(mu);
        err = "device status " + std::to_string(s.h->status.code) + " at (" +
              std::to_string(s.h->status.where[0]) + ", " + std::to_string(s.h->status.where[1]) +
              ", " + std::to_string(s.h->status.where[2]) + ")";
    }
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        Request *r = s.reqs[i];
        ara_status st = group_st;
        const double *o = s.h->out + i * 2 * ARA_SERVER_MAX_RP;
        const size_t n_rp = r->rps.size();
        for (size_t k = 0; k < n_rp && st == ARA_OK; ++k) {
            r->res.pml[k] = o[k];
            r->res.tvar[k] = o[n_rp + k];
        }
        if (st == ARA_OK && r->want_ylt) {
            const char *yp = pool + r->off + r->ws_bytes + r->ylt_l_bytes;
            r->ylt_host.resize((size_t)r->trial_count);
            if (hipMemcpyAsync(r->ylt_host.data(), yp, sizeof(float) * r->ylt_host.size(),
                               hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
                hipStreamSynchronize(s.stream) != hipSuccess)
                st = ARA_E_HIP;
            r->res.ylt = r->ylt_host.data();
            r->res.ylt_count = (int64_t)r->ylt_host.size();
        }
        finish(r, st);
    }
    s.reqs.clear();
    s.busy = false;
    return true;
}

void ara_server::run() {
    (void)hipSetDevice(device);
    const size_t ready_cap = (size_t)cfg.max_batch * (size_t)cfg.max_inflight;
    while (true) {
        bool did = false;
        for (Slot &s : slots) did = complete(s) || did;
        for (Slot &s : slots)
            if (!s.busy) did = launch(s) || did;
        if (ready.size() < ready_cap) did = load_one() || did;
        std::unique_lock<std::mutex> lk(mu);
        bool any_busy = false;
        for (Slot &s : slots) any_busy = any_busy || s.busy;
        if (stop && pending.empty() && ready.empty() && !any_busy) break;
        if (!did) {
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
}

void ara_server::destroy_all() {
    for (Slot &s : slots) {
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.d_status) (void)hipFree(s.d_status);
        if (s.h) (void)hipHostFree(s.h);
        s = Slot();
    }
    if (load_stream) (void)hipStreamDestroy(load_stream);
    load_stream = nullptr;
    if (ctx) ara_destroy(ctx);            // frees the YET registration and any portfolios
    ctx = nullptr;
    delete alloc;
    alloc = nullptr;
}

extern "C" {

ara_status ara_server_create(int hip_device, int64_t n_trials, int32_t n_catalogue,
                             const int64_t *d_trial_offsets, const int32_t *d_event_ids,
                             const ara_server_config *cfg, ara_server **out) {
    if (!out || !cfg || !cfg->d_pool || cfg->pool_bytes == 0 || n_trials <= 0 || n_catalogue <= 0)
        return ARA_E_INVALID_ARG;
    if (cfg->sum_mode != ARA_SUM_NAIVE32 && cfg->sum_mode != ARA_SUM_KAHAN32 &&
        cfg->sum_mode != ARA_SUM_F64)
        return ARA_E_INVALID_ARG;
    *out = nullptr;
    ara_server *srv = new ara_server();
    srv->cfg = *cfg;
    if (srv->cfg.max_inflight <= 0) srv->cfg.max_inflight = 2;
    if (srv->cfg.max_batch <= 0) srv->cfg.max_batch = 4;
    srv->device = hip_device;
    srv->pool = (char *)cfg->d_pool;
    srv->n_catalogue = n_catalogue;
    srv->n_trials = n_trials;
    const size_t sb = slot_scratch_bytes(srv->cfg.max_batch, n_trials);
    const size_t all_sb = sb * (size_t)srv->cfg.max_inflight;
    if (all_sb >= cfg->pool_bytes) {
        delete srv;
        return ARA_E_WORKSPACE_TOO_SMALL;
    }
    srv->alloc = new PoolAllocator(cfg->pool_bytes);
    srv->request_room = cfg->pool_bytes - all_sb;
    ara_status st = ara_create(hip_device, &srv->ctx);
    if (st == ARA_OK)
        st = ara_load_yet(srv->ctx, n_trials, n_catalogue, d_trial_offsets, d_event_ids, nullptr,
                          nullptr, &srv->yet);
    if (st == ARA_OK && hipStreamCreate(&srv->load_stream) != hipSuccess) st = ARA_E_HIP;
    srv->slots.resize((size_t)srv->cfg.max_inflight);
    const size_t hb = sizeof(HostBlock) +
                      sizeof(double) * 2 * ARA_SERVER_MAX_RP * (size_t)srv->cfg.max_batch;
    for (Slot &s : srv->slots) {
        if (st != ARA_OK) break;
        if (!srv->alloc->alloc(sb, &s.scratch_off)) {
            st = ARA_E_WORKSPACE_TOO_SMALL;
            break;
        }
        s.scratch_bytes = sb;
        if (hipStreamCreate(&s.stream) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&s.d_status, sizeof(ara::Status)) != hipSuccess ||
            hipHostMalloc((void **)&s.h, hb, hipHostMallocDefault) != hipSuccess)
            st = ARA_E_HIP;
    }
    if (st != ARA_OK) {
        srv->destroy_all();
        delete srv;
        return st;
    }
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return ARA_OK;
}

ara_status ara_server_submit(ara_server *srv, const ara_portfolio_desc *desc, int64_t trial_begin,
                             int64_t trial_count, const double *return_periods, int32_t n_rp,
                             int32_t flags, uint64_t *request_id) {
    if (!srv || !desc || !return_periods || n_rp <= 0 || n_rp > ARA_SERVER_MAX_RP ||
        (flags & ~(ARA_SUBMIT_WANT_YLT | ARA_SUBMIT_BORROW)) ||
        trial_begin < 0 || trial_count <= 0 || trial_begin + trial_count > srv->n_trials ||
        desc->n_layers < 0 || (desc->n_layers > 0 && !desc->layers))
        return ARA_E_INVALID_ARG;
    for (int32_t i = 0; i < n_rp; ++i)
        if (!(return_periods[i] > 0.0)) return ARA_E_INVALID_ARG;
    for (int l = 0; l < desc->n_layers; ++l) {
        const ara_layer_desc &L = desc->layers[l];
        if (L.n_elts < 0 || (L.n_elts > 0 && !L.elts)) return ARA_E_INVALID_ARG;
        for (int j = 0; j < L.n_elts; ++j) {
            const ara_elt_desc &e = L.elts[j];
            if (e.n_rows < 0 || (e.n_rows > 0 && (!e.event_ids || !e.mean)))
                return ARA_E_INVALID_ARG;
        }
    }
    Request *r = new Request();
    const int nl = desc->n_layers;
    r->layers.resize((size_t)nl);
    r->elts.resize((size_t)nl);
    for (int l = 0; l < nl; ++l) {
        const ara_layer_desc &L = desc->layers[l];
        r->layers[l] = L;
        r->elts[l].resize((size_t)L.n_elts);
        for (int j = 0; j < L.n_elts; ++j) {
            const ara_elt_desc &e = L.elts[j];
            const size_t n = (size_t)e.n_rows;
            ara_elt_desc c = e;             // borrowed: the caller's row arrays
            if (!(flags & ARA_SUBMIT_BORROW)) {
                auto copyf = [&](std::vector<std::vector<float>> &dst,
                                 const float *src) -> const float * {
                    if (!src) return nullptr;
                    dst.emplace_back(src, src + n);
                    return dst.back().data();
                };
                r->ev.emplace_back(e.event_ids, e.event_ids + n);
                c.event_ids = r->ev.back().data();
                c.mean = copyf(r->mean, e.mean);
                c.sigma_i = copyf(r->si, e.sigma_i);
                c.sigma_c = copyf(r->sc, e.sigma_c);
                c.max_loss = copyf(r->mx, e.max_loss);
            }
            r->elts[l][j] = c;
        }
        r->layers[l].elts = r->elts[l].data();
    }
    r->desc = *desc;
    r->desc.layers = r->layers.data();
    r->trial_begin = trial_begin;
    r->trial_count = trial_count;
    r->rps.assign(return_periods, return_periods + n_rp);
    metric_ranks(r);
    r->want_ylt = (flags & ARA_SUBMIT_WANT_YLT) ? 1 : 0;
    ara_status st = request_footprint(srv, r);
    if (st != ARA_OK) {
        delete r;
        return st;
    }
    if (r->footprint > srv->request_room) {
        delete r;
        return ARA_E_WORKSPACE_TOO_SMALL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    r->id = srv->next_id++;
    r->t_submit = Clock::now();
    if (request_id) *request_id = r->id;
    srv->pending.push_back(r);
    srv->cv_work.notify_one();
    return ARA_OK;
}

ara_status ara_server_poll(ara_server *srv, ara_server_result *out, int32_t max_results,
                           double wait_s, int32_t *n_out) {
    if (!srv || !out || max_results <= 0 || !n_out) return ARA_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->finished.empty() && wait_s > 0)
        srv->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s),
                              [srv] { return !srv->finished.empty(); });
    int32_t n = 0;
    while (n < max_results && !srv->finished.empty()) {
        Request *r = srv->finished.front();
        srv->finished.pop_front();
        out[n++] = r->res;
        srv->handed_out[r->id] = r;
    }
    *n_out = n;
    return ARA_OK;
}

ara_status ara_server_release(ara_server *srv, uint64_t request_id) {
    if (!srv) return ARA_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->handed_out.find(request_id);
    if (it == srv->handed_out.end()) return ARA_E_INVALID_ARG;
    delete it->second;
    srv->handed_out.erase(it);
    return ARA_OK;
}

ara_status ara_server_destroy(ara_server *srv) {
    if (!srv) return ARA_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (Request *r : srv->finished) delete r;
    for (auto &kv : srv->handed_out) delete kv.second;
    srv->destroy_all();
    delete srv;
    return ARA_OK;
}

const char *ara_server_last_error(ara_server *srv) {
    if (!srv) return "no server";
    std::lock_guard<std::mutex> lk(srv->mu);
    thread_local std::string copy;
    copy = srv->err;
    return copy.c_str();
}

}  // extern "C"
