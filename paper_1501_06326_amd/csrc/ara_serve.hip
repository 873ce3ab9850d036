// ara_serve.hip -- serving loop: a YET resident in HBM, portfolio-pricing
// requests admitted by HBM footprint and run in batched launches that overlap
// on the device (continuous batching), PML / TVaR and latencies on completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
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

// A request with its own copy of the portfolio description.
struct Request {
    uint64_t id = 0;
    std::vector<std::vector<int32_t>> ev;
    std::vector<std::vector<float>> mean, si, sc, mx;
    std::vector<std::vector<ara_elt_desc>> elts;
    std::vector<ara_layer_desc> layers;
    ara_portfolio_desc desc{};
    int64_t trial_begin = 0, trial_count = 0;
    std::vector<double> rps;
    int want_ylt = 0;
    size_t ws_bytes = 0, ylt_l_bytes = 0, ylt_p_bytes = 0, pml_bytes = 0, footprint = 0;
    size_t off = 0;                    // pool offset of the allocation
    ara_portfolio *pf = nullptr;
    Clock::time_point t_submit, t_launch, t_done;
    ara_server_result res{};
    std::vector<float> ylt_host;
};

// One stream of the continuous batch.  Each slot owns an ara_context (its own
// device status word) and its own registration of the shared YET, so that the
// validation of a request being loaded on one slot never reads or clears an
// error raised by a launch still running on another.
struct Slot {
    ara_context *ctx = nullptr;
    ara_yet *yet = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    size_t scratch_off = 0, scratch_bytes = 0;
};

}  // namespace

struct ara_server {
    int device = 0;
    ara_server_config cfg{};
    char *pool = nullptr;
    PoolAllocator *alloc = nullptr;
    int32_t n_catalogue = 0;
    int64_t n_trials = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::deque<Request *> finished;
    std::map<uint64_t, Request *> released_wait;   // results handed out, not yet released
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    std::string err;

    void run();
    void finalize(Slot &s);
    void launch_group(Slot &s, std::vector<Request *> &group);
    bool admit(std::vector<Request *> &group, size_t *scratch_off, size_t *scratch_bytes);
    void destroy_slots();
};

namespace {

ara_status request_footprint(ara_server *srv, Request *r) {
    size_t ws = 0;
    ara_status st = ara_portfolio_workspace_size(&r->desc, srv->n_catalogue, &ws);
    if (st != ARA_OK) return st;
    size_t pml = 0;
    ara_pml_tvar_scratch_size(r->trial_count, &pml);
    r->ws_bytes = align_up(ws);
    r->ylt_l_bytes = align_up(sizeof(float) * (size_t)r->desc.n_layers * (size_t)r->trial_count);
    r->ylt_p_bytes = align_up(sizeof(float) * (size_t)r->trial_count);
    r->pml_bytes = align_up(pml);
    r->footprint = r->ws_bytes + r->ylt_l_bytes + r->ylt_p_bytes + r->pml_bytes;
    return ARA_OK;
}

}  // namespace

// Takes requests from the head of the queue while their footprints fit in the
// pool (arrival order: a request that does not fit holds back those behind it),
// then the batch scratch for the group; if the scratch does not fit the
// youngest request goes back to the queue and the group shrinks.  Called with
// the lock held.
bool ara_server::admit(std::vector<Request *> &group, size_t *scratch_off,
                       size_t *scratch_bytes) {
    while (!pending.empty() && (int)group.size() < cfg.max_batch) {
        Request *r = pending.front();
        size_t off;
        if (!alloc->alloc(r->footprint, &off)) break;
        r->off = off;
        group.push_back(r);
        pending.pop_front();
    }
    while (!group.empty()) {
        int64_t maxc = 0;
        for (Request *r : group) maxc = std::max(maxc, r->trial_count);
        const size_t sb = ara::batch_scratch_need((int32_t)group.size(), maxc);
        if (alloc->alloc(sb, scratch_off)) {
            *scratch_bytes = sb;
            return true;
        }
        Request *r = group.back();
        group.pop_back();
        alloc->release(r->off, r->footprint);
        pending.push_front(r);
    }
    return false;
}

// Loads each request's portfolio tables into its pool region (host-side and
// device-side validation; a request that fails there fails alone) and enqueues
// one batched launch for the rest of the group on the slot's stream.
void ara_server::launch_group(Slot &s, std::vector<Request *> &group) {
    std::vector<ara_portfolio *> pfs;
    std::vector<void *> yl, yp;
    std::vector<int64_t> ranges;
    for (Request *r : group) {
        char *base = pool + r->off;
        r->t_launch = Clock::now();
        ara_status st = ara_load_portfolio(s.ctx, &r->desc, n_catalogue, base, r->ws_bytes,
                                           s.stream, &r->pf);
        r->res.status = st;
        if (st != ARA_OK) {
            r->pf = nullptr;
            std::lock_guard<std::mutex> lk(mu);
            err = "request " + std::to_string(r->id) + ": " + ara_last_error(s.ctx);
            continue;
        }
        pfs.push_back(r->pf);
        yl.push_back(base + r->ws_bytes);
        yp.push_back(base + r->ws_bytes + r->ylt_l_bytes);
        ranges.push_back(r->trial_begin);
        ranges.push_back(r->trial_count);
    }
    if (!pfs.empty()) {
        ara_run_opts o;
        std::memset(&o, 0, sizeof o);
        o.sum_mode = cfg.sum_mode;
        o.ylt_dtype = ARA_F32;
        ara_status st = ara::run_batch_ranges(s.ctx, s.yet, (int32_t)pfs.size(), pfs.data(), &o,
                                              nullptr, yl.data(), yp.data(), ranges.data(),
                                              pool + s.scratch_off, s.scratch_bytes, s.stream);
        if (st != ARA_OK)
            for (Request *r : group)
                if (r->pf) r->res.status = st;
    }
    if (hipEventRecord(s.done, s.stream) != hipSuccess) {
        // without the event the slot cannot be polled: finish it synchronously
        (void)hipStreamSynchronize(s.stream);
        for (Request *r : group)
            if (r->res.status == ARA_OK) r->res.status = ARA_E_HIP;
    }
    s.reqs = group;
    s.busy = true;
}

void ara_server::finalize(Slot &s) {
    // the batched launch's device status covers the whole group
    const ara_status group_st = ara_sync_status(s.ctx, s.stream);
    for (Request *r : s.reqs) {
        char *base = pool + r->off;
        if (r->res.status == ARA_OK) {
            const float *yp = (const float *)(base + r->ws_bytes + r->ylt_l_bytes);
            ara_status st = group_st;
            if (st == ARA_OK && r->trial_count > 0)
                st = ara_pml_tvar(s.ctx, yp, ARA_F32, r->trial_count, r->rps.data(),
                                  (int32_t)r->rps.size(), r->res.pml, r->res.tvar,
                                  base + r->ws_bytes + r->ylt_l_bytes + r->ylt_p_bytes,
                                  r->pml_bytes, s.stream);
            if (st == ARA_OK && r->want_ylt) {
                r->ylt_host.resize((size_t)r->trial_count);
                if (hipMemcpyAsync(r->ylt_host.data(), yp, sizeof(float) * r->ylt_host.size(),
                                   hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
                    hipStreamSynchronize(s.stream) != hipSuccess)
                    st = ARA_E_HIP;
                r->res.ylt = r->ylt_host.data();
                r->res.ylt_count = (int64_t)r->ylt_host.size();
            }
            r->res.status = st;
        }
        if (r->res.status != ARA_OK) {
            std::lock_guard<std::mutex> lk(mu);
            err = "request " + std::to_string(r->id) + ": " + ara_last_error(s.ctx);
        }
        if (r->pf) ara_free_portfolio(s.ctx, r->pf);
        r->pf = nullptr;
        r->t_done = Clock::now();
        r->res.request_id = r->id;
        r->res.n_rp = (int32_t)r->rps.size();
        r->res.queue_s = seconds_since(r->t_submit, r->t_launch);
        r->res.latency_s = seconds_since(r->t_submit, r->t_done);
    }
    std::lock_guard<std::mutex> lk(mu);
    for (Request *r : s.reqs) {
        alloc->release(r->off, r->footprint);
        finished.push_back(r);
    }
    alloc->release(s.scratch_off, s.scratch_bytes);
    s.reqs.clear();
    s.busy = false;
    cv_done.notify_all();
}

void ara_server::destroy_slots() {
    for (Slot &s : slots) {
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.ctx) ara_destroy(s.ctx);       // frees the slot's YET registration too
        s = Slot();
    }
}

void ara_server::run() {
    (void)hipSetDevice(device);
    while (true) {
        bool did = false;
        // completions
        for (Slot &s : slots)
            if (s.busy && hipEventQuery(s.done) == hipSuccess) {
                finalize(s);
                did = true;
            }
        // admission: requests in arrival order while the pool and a stream allow
        for (Slot &s : slots) {
            if (s.busy) continue;
            std::vector<Request *> group;
            bool ok;
            {
                std::lock_guard<std::mutex> lk(mu);
                ok = admit(group, &s.scratch_off, &s.scratch_bytes);
            }
            if (!ok) break;
            launch_group(s, group);
            did = true;
        }
        std::unique_lock<std::mutex> lk(mu);
        bool any_busy = false;
        for (Slot &s : slots) any_busy = any_busy || s.busy;
        if (stop && pending.empty() && !any_busy) break;
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
    if (srv->cfg.max_inflight <= 0) srv->cfg.max_inflight = 4;
    if (srv->cfg.max_batch <= 0) srv->cfg.max_batch = 16;
    srv->device = hip_device;
    srv->pool = (char *)cfg->d_pool;
    srv->alloc = new PoolAllocator(cfg->pool_bytes);
    srv->n_catalogue = n_catalogue;
    srv->n_trials = n_trials;
    srv->slots.resize((size_t)srv->cfg.max_inflight);
    ara_status st = ARA_OK;
    for (Slot &s : srv->slots) {
        st = ara_create(hip_device, &s.ctx);
        if (st == ARA_OK)
            st = ara_load_yet(s.ctx, n_trials, n_catalogue, d_trial_offsets, d_event_ids, nullptr,
                              nullptr, &s.yet);
        if (st == ARA_OK && (hipStreamCreate(&s.stream) != hipSuccess ||
                             hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess))
            st = ARA_E_HIP;
        if (st != ARA_OK) break;
    }
    if (st != ARA_OK) {
        srv->destroy_slots();
        delete srv->alloc;
        delete srv;
        return st;
    }
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return ARA_OK;
}

ara_status ara_server_submit(ara_server *srv, const ara_portfolio_desc *desc, int64_t trial_begin,
                             int64_t trial_count, const double *return_periods, int32_t n_rp,
                             int32_t want_ylt, uint64_t *request_id) {
    if (!srv || !desc || !return_periods || n_rp <= 0 || n_rp > ARA_SERVER_MAX_RP ||
        trial_begin < 0 || trial_count <= 0 || trial_begin + trial_count > srv->n_trials)
        return ARA_E_INVALID_ARG;
    Request *r = new Request();
    const int nl = desc->n_layers;
    r->layers.resize((size_t)(nl > 0 ? nl : 0));
    r->elts.resize((size_t)(nl > 0 ? nl : 0));
    for (int l = 0; l < nl; ++l) {
        const ara_layer_desc &L = desc->layers[l];
        r->layers[l] = L;
        r->elts[l].resize((size_t)(L.n_elts > 0 ? L.n_elts : 0));
        for (int j = 0; j < L.n_elts; ++j) {
            const ara_elt_desc &e = L.elts[j];
            const size_t n = (size_t)(e.n_rows > 0 ? e.n_rows : 0);
            auto copyf = [&](std::vector<std::vector<float>> &dst, const float *src) -> const float * {
                if (!src) return nullptr;
                dst.emplace_back(src, src + n);
                return dst.back().data();
            };
            ara_elt_desc c = e;
            r->ev.emplace_back(e.event_ids, e.event_ids + n);
            c.event_ids = r->ev.back().data();
            c.mean = copyf(r->mean, e.mean);
            c.sigma_i = copyf(r->si, e.sigma_i);
            c.sigma_c = copyf(r->sc, e.sigma_c);
            c.max_loss = copyf(r->mx, e.max_loss);
            r->elts[l][j] = c;
        }
        r->layers[l].elts = r->elts[l].data();
    }
    r->desc = *desc;
    r->desc.layers = r->layers.data();
    r->trial_begin = trial_begin;
    r->trial_count = trial_count;
    r->rps.assign(return_periods, return_periods + n_rp);
    r->want_ylt = want_ylt;
    ara_status st = request_footprint(srv, r);
    if (st != ARA_OK) {
        delete r;
        return st;
    }
    const size_t group_scratch = ara::batch_scratch_need(1, trial_count);
    if (r->footprint + align_up(group_scratch) > srv->cfg.pool_bytes) {
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
        srv->released_wait[r->id] = r;
    }
    *n_out = n;
    return ARA_OK;
}

ara_status ara_server_release(ara_server *srv, uint64_t request_id) {
    if (!srv) return ARA_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->released_wait.find(request_id);
    if (it == srv->released_wait.end()) return ARA_E_INVALID_ARG;
    delete it->second;
    srv->released_wait.erase(it);
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
    srv->destroy_slots();
    for (Request *r : srv->finished) delete r;
    for (auto &kv : srv->released_wait) delete kv.second;
    delete srv->alloc;
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
