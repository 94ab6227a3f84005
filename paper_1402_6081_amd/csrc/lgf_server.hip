// Request server: many independent solves u = G * f (Sec. 3.1 per request) served from one
// process on one GPU.  A dispatcher thread takes requests in arrival order, admits each one
// when a stream slot is free and its plan fits the HBM budget, runs it on the slot's
// stream and retires it when the slot's completion event has fired.
//
// Residency: plans (lists and workspace) are cached by layout and reused by later requests
// of the same layout; kernel spectra live in the library-wide cache keyed by (n, p, level,
// precision), so they are shared by every plan.  When a new plan does not fit the budget,
// idle cached plans are evicted in least-recently-used order; if it still does not fit, the
// head of the queue waits until running requests release their plans.  A plan serves one
// request at a time (one workspace); a second concurrent request of the same layout gets a
// second plan instance if the budget allows, else it waits.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_internal.h"

using namespace lgfdev;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct CachedPlan {
    std::string key;
    lgf_plan_t plan = nullptr;
    int64_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

struct Request {
    int64_t ticket = 0;
    std::vector<int32_t> layout;
    std::string key;
    int64_t nblocks = 0;
    const void* f = nullptr;
    void* u = nullptr;
    // recorded on the submitter's stream at submit time: the slot stream waits for it, so the
    // solve reads f (and overwrites u) only after the work the caller queued before submit
    hipEvent_t ev_ready = nullptr;
    Clock::time_point t_submit, t_start, t_done;
    lgf_status status = LGF_OK;
    std::string error;
    bool done = false;
    int slot = -1;
    CachedPlan* cp = nullptr;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    double device_ms = 0.0;
};

std::string layout_key(const int32_t* ijk, int64_t nb) {
    std::string k(reinterpret_cast<const char*>(ijk), (size_t)nb * 3 * sizeof(int32_t));
    return k;
}

}  // namespace

struct lgf_server_s {
    lgf_server_config cfg{};
    int device = 0;
    int spectra_mode = 0;  // kernel spectra of the server's plans: the process-wide mode at creation
    std::vector<hipStream_t> slots;
    std::vector<bool> slot_busy;
    std::vector<hipEvent_t> ev_pool;
    std::vector<hipEvent_t> ready_pool;  // submit-time events (shared with submitting threads, under mu)

    std::mutex mu;
    std::condition_variable cv_work;  // new request or shutdown
    std::condition_variable cv_done;  // a request finished
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int64_t, std::shared_ptr<Request>> tickets;
    int64_t next_ticket = 1;
    bool stop = false;

    // dispatcher-owned state
    std::vector<std::shared_ptr<Request>> inflight;
    std::list<std::unique_ptr<CachedPlan>> plans;
    int64_t plan_bytes = 0;
    uint64_t use_clock = 0;

    // statistics (under mu)
    std::vector<double> latencies_ms;
    int64_t completed = 0, failed = 0, points = 0, plans_created = 0, plans_evicted = 0;
    Clock::time_point t_first_submit, t_last_done;
    bool any_submit = false;

    std::thread worker;

    ~lgf_server_s() {
        for (auto& cp : plans) lgf_plan_destroy(cp->plan);
        for (auto e : ev_pool) hipEventDestroy(e);
        for (auto e : ready_pool) hipEventDestroy(e);
        for (auto s : slots) hipStreamDestroy(s);
    }
};

namespace {

hipEvent_t take_event(lgf_server_s* S) {
    if (!S->ev_pool.empty()) {
        hipEvent_t e = S->ev_pool.back();
        S->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void finish(lgf_server_s* S, const std::shared_ptr<Request>& r, lgf_status st, const std::string& err) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (r->ev_ready) {
        S->ready_pool.push_back(r->ev_ready);
        r->ev_ready = nullptr;
    }
    r->status = st;
    r->error = err;
    r->done = true;
    r->t_done = Clock::now();
    if (st == LGF_OK) {
        ++S->completed;
        S->points += r->nblocks * (int64_t)S->cfg.n * S->cfg.n * S->cfg.n;
        S->latencies_ms.push_back(ms_between(r->t_submit, r->t_done));
        S->t_last_done = r->t_done;
    } else {
        ++S->failed;
    }
    S->cv_done.notify_all();
}

// Retire requests whose completion event has fired.  Returns true if any did.
bool retire(lgf_server_s* S) {
    bool any = false;
    for (size_t i = 0; i < S->inflight.size();) {
        auto r = S->inflight[i];
        const hipError_t q = hipEventQuery(r->ev_end);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (q == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r->ev_start, r->ev_end) == hipSuccess) r->device_ms = ms;
        }
        r->cp->busy = false;
        r->cp->last_use = ++S->use_clock;
        S->slot_busy[r->slot] = false;
        S->ev_pool.push_back(r->ev_start);
        S->ev_pool.push_back(r->ev_end);
        S->inflight[i] = S->inflight.back();
        S->inflight.pop_back();
        finish(S, r, q == hipSuccess ? LGF_OK : LGF_ERR_DEVICE,
               q == hipSuccess ? std::string() : std::string("solve failed: ") + hipGetErrorString(q));
        any = true;
    }
    return any;
}

int64_t resident_bytes(lgf_server_s* S) { return S->plan_bytes + spectra_bytes_total(); }

// Try to start the request at the head of the queue.  Returns 1 if started or failed
// (the queue advanced), 0 if it has to wait.
int try_admit(lgf_server_s* S, const std::shared_ptr<Request>& r) {
    int slot = -1;
    for (size_t k = 0; k < S->slots.size(); ++k)
        if (!S->slot_busy[k]) {
            slot = (int)k;
            break;
        }
    if (slot < 0) return 0;
    CachedPlan* cp = nullptr;
    for (auto& c : S->plans)
        if (!c->busy && c->key == r->key) {
            cp = c.get();
            break;
        }
    if (!cp) {
        int64_t est = 0;
        lgf_status st = plan_estimate(r->layout.data(), r->nblocks, S->cfg.n, S->cfg.p, S->cfg.levels,
                                      (lgf_precision)S->cfg.precision, &est);
        if (st != LGF_OK) {
            finish(S, r, st, lgf_last_error());
            return 1;
        }
        const int64_t budget = S->cfg.budget_bytes;
        if (budget > 0 && est + spectra_bytes_total() > budget) {
            finish(S, r, LGF_ERR_BUDGET, "request exceeds the server's HBM budget on its own");
            return 1;
        }
        // evict idle plans, least recently used first, until the new one fits
        while (budget > 0 && resident_bytes(S) + est > budget) {
            auto victim = S->plans.end();
            for (auto it = S->plans.begin(); it != S->plans.end(); ++it)
                if (!(*it)->busy && (victim == S->plans.end() || (*it)->last_use < (*victim)->last_use)) victim = it;
            if (victim == S->plans.end()) break;
            S->plan_bytes -= (*victim)->bytes;
            lgf_plan_destroy((*victim)->plan);
            S->plans.erase(victim);
            std::lock_guard<std::mutex> lk(S->mu);
            ++S->plans_evicted;
        }
        if (budget > 0 && resident_bytes(S) + est > budget) return 0;  // wait for running work
        lgf_plan_t pl = nullptr;
        st = lgf_plan_create(r->layout.data(), r->nblocks, S->cfg.n, S->cfg.p, S->cfg.levels,
                             (lgf_precision)S->cfg.precision, S->slots[slot], &pl);
        if (st != LGF_OK) {
            finish(S, r, st, lgf_last_error());
            return 1;
        }
        lgf_plan_info info;
        lgf_plan_query(pl, &info);
        auto c = std::make_unique<CachedPlan>();
        c->key = r->key;
        c->plan = pl;
        c->bytes = info.workspace_bytes;
        cp = c.get();
        S->plans.push_back(std::move(c));
        S->plan_bytes += cp->bytes;
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->plans_created;
    }
    r->ev_start = take_event(S);
    r->ev_end = take_event(S);
    if (!r->ev_start || !r->ev_end) {
        finish(S, r, LGF_ERR_DEVICE, "event creation failed");
        return 1;
    }
    hipStream_t s = S->slots[slot];
    r->t_start = Clock::now();
    // the solve follows everything the submitter had queued on its stream before the submit
    if (hipStreamWaitEvent(s, r->ev_ready, 0) != hipSuccess) {
        S->ev_pool.push_back(r->ev_start);
        S->ev_pool.push_back(r->ev_end);
        finish(S, r, LGF_ERR_DEVICE, "stream wait on the submit event failed");
        return 1;
    }
    hipEventRecord(r->ev_start, s);
    lgf_status st = lgf_solve(cp->plan, r->f, r->u, s);
    hipEventRecord(r->ev_end, s);
    if (st != LGF_OK) {
        S->ev_pool.push_back(r->ev_start);
        S->ev_pool.push_back(r->ev_end);
        finish(S, r, st, lgf_last_error());
        return 1;
    }
    cp->busy = true;
    r->cp = cp;
    r->slot = slot;
    S->slot_busy[slot] = true;
    S->inflight.push_back(r);
    return 1;
}

void dispatcher(lgf_server_s* S) {
    hipSetDevice(S->device);
    lgfdev::spectra_set_thread_mode(S->spectra_mode);  // the plans this thread creates
    for (;;) {
        retire(S);
        std::shared_ptr<Request> head;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->queue.empty()) {
                if (S->stop && S->inflight.empty()) return;
                if (S->inflight.empty()) {
                    S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
                    continue;
                }
            } else {
                head = S->queue.front();
            }
        }
        int advanced = 0;
        if (head) {
            advanced = try_admit(S, head);
            if (advanced) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->queue.pop_front();
            }
        }
        // nothing to start: poll the running requests' events
        if (!advanced && !S->inflight.empty()) std::this_thread::yield();
    }
}

}  // namespace

extern "C" {

lgf_status lgf_server_create(const lgf_server_config* cfg, lgf_server_t* out) {
    if (!out || !cfg) {
        set_last_error("NULL argument to lgf_server_create");
        return LGF_ERR_ARG;
    }
    *out = nullptr;
    if (cfg->n != 4 && cfg->n != 8 && cfg->n != 16) {
        set_last_error("n must be 4, 8 or 16");
        return LGF_ERR_ARG;
    }
    if (cfg->p < 2 || (cfg->p > 10 && !(cfg->n == 16 && cfg->p == 17)) ||
        (cfg->precision != LGF_F64 && cfg->precision != LGF_F32) ||
        cfg->max_slots < 1 || cfg->max_slots > 16 || cfg->budget_bytes < 0 || cfg->max_queue < 0) {
        set_last_error("lgf_server_create: p in [2, 10] (or 17 with n = 16), precision, max_slots in [1, 16], budget >= 0");
        return LGF_ERR_ARG;
    }
    auto S = std::make_unique<lgf_server_s>();
    S->cfg = *cfg;
    S->spectra_mode = lgfdev::spectra_mode();
    if (hipGetDevice(&S->device) != hipSuccess) {
        set_last_error("no HIP device");
        return LGF_ERR_DEVICE;
    }
    for (int k = 0; k < cfg->max_slots; ++k) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            set_last_error("stream creation failed");
            return LGF_ERR_DEVICE;
        }
        S->slots.push_back(s);
        S->slot_busy.push_back(false);
    }
    lgf_server_s* raw = S.release();
    raw->worker = std::thread(dispatcher, raw);
    *out = raw;
    return LGF_OK;
}

lgf_status lgf_server_submit(lgf_server_t S, const int32_t* block_ijk, int64_t nblocks, const void* f, void* u,
                             void* hip_stream, int64_t* ticket) {
    if (!S || !block_ijk || !f || !u || !ticket || nblocks < 1) {
        set_last_error("bad arguments to lgf_server_submit");
        return LGF_ERR_ARG;
    }
    auto r = std::make_shared<Request>();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->ready_pool.empty()) {
            r->ev_ready = S->ready_pool.back();
            S->ready_pool.pop_back();
        }
    }
    if (!r->ev_ready && hipEventCreateWithFlags(&r->ev_ready, hipEventDisableTiming) != hipSuccess) {
        r->ev_ready = nullptr;
        set_last_error("event creation failed in lgf_server_submit");
        return LGF_ERR_DEVICE;
    }
    auto give_back = [&]() {
        std::lock_guard<std::mutex> lk(S->mu);
        S->ready_pool.push_back(r->ev_ready);
        r->ev_ready = nullptr;
    };
    if (hipEventRecord(r->ev_ready, (hipStream_t)hip_stream) != hipSuccess) {
        give_back();
        set_last_error("lgf_server_submit: recording on the caller's stream failed");
        return LGF_ERR_DEVICE;
    }
    r->layout.assign(block_ijk, block_ijk + 3 * nblocks);
    r->key = layout_key(block_ijk, nblocks);
    r->nblocks = nblocks;
    r->f = f;
    r->u = u;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            S->ready_pool.push_back(r->ev_ready);
            set_last_error("server is shutting down");
            return LGF_ERR_ARG;
        }
        if (S->cfg.max_queue > 0 && (int64_t)S->queue.size() >= S->cfg.max_queue) {
            S->ready_pool.push_back(r->ev_ready);
            set_last_error("request queue is full");
            return LGF_ERR_BUSY;
        }
        r->ticket = S->next_ticket++;
        S->queue.push_back(r);
        S->tickets[r->ticket] = r;
        if (!S->any_submit) {
            S->any_submit = true;
            S->t_first_submit = r->t_submit;
        }
    }
    S->cv_work.notify_one();
    *ticket = r->ticket;
    return LGF_OK;
}

static void fill_result(const Request& r, lgf_request_result* res) {
    if (!res) return;
    std::memset(res, 0, sizeof(*res));
    res->status = r.status;
    res->latency_ms = ms_between(r.t_submit, r.t_done);
    res->queue_ms = r.t_start.time_since_epoch().count() ? ms_between(r.t_submit, r.t_start) : 0.0;
    res->device_ms = r.device_ms;
    res->nblocks = r.nblocks;
}

lgf_status lgf_server_poll(lgf_server_t S, int64_t ticket, int32_t* done, lgf_request_result* res) {
    if (!S || !done) {
        set_last_error("bad arguments to lgf_server_poll");
        return LGF_ERR_ARG;
    }
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->tickets.find(ticket);
        if (it == S->tickets.end()) {
            set_last_error("unknown ticket");
            return LGF_ERR_ARG;
        }
        r = it->second;
        *done = r->done ? 1 : 0;
        if (!r->done) return LGF_OK;
        S->tickets.erase(it);
    }
    fill_result(*r, res);
    if (r->status != LGF_OK) set_last_error(r->error);
    return LGF_OK;
}

lgf_status lgf_server_wait(lgf_server_t S, int64_t ticket, lgf_request_result* res) {
    if (!S) {
        set_last_error("NULL server");
        return LGF_ERR_ARG;
    }
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->tickets.find(ticket);
        if (it == S->tickets.end()) {
            set_last_error("unknown ticket");
            return LGF_ERR_ARG;
        }
        r = it->second;
        S->cv_done.wait(lk, [&] { return r->done; });
        S->tickets.erase(ticket);
    }
    fill_result(*r, res);
    if (r->status != LGF_OK) set_last_error(r->error);
    return LGF_OK;
}

lgf_status lgf_server_stats(lgf_server_t S, lgf_server_stats_t* out) {
    if (!S || !out) {
        set_last_error("bad arguments to lgf_server_stats");
        return LGF_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->completed = S->completed;
    out->failed = S->failed;
    out->queued = (int64_t)S->queue.size();
    out->points = S->points;
    out->plans_created = S->plans_created;
    out->plans_evicted = S->plans_evicted;
    out->plan_bytes = S->plan_bytes;
    out->spectra_bytes = spectra_bytes_total();
    if (!S->latencies_ms.empty()) {
        std::vector<double> v = S->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double fr = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1.0 - fr) + v[i + 1] * fr : v[i];
        };
        out->latency_p50_ms = pct(0.50);
        out->latency_p99_ms = pct(0.99);
        out->latency_max_ms = v.back();
        const double span = ms_between(S->t_first_submit, S->t_last_done);
        out->points_per_s = span > 0 ? (double)S->points / (span * 1e-3) : 0.0;
    }
    return LGF_OK;
}

lgf_status lgf_server_reset_stats(lgf_server_t S) {
    if (!S) {
        set_last_error("NULL server");
        return LGF_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->latencies_ms.clear();
    S->completed = S->failed = S->points = 0;
    S->any_submit = false;
    return LGF_OK;
}

lgf_status lgf_server_destroy(lgf_server_t S) {
    if (!S) return LGF_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto s : S->slots) hipStreamSynchronize(s);
    delete S;
    return LGF_OK;
}

}  // extern "C"
