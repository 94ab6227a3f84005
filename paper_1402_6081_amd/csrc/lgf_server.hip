// Request server: many independent solves u = G * f (Sec. 3.1 per request) served from one
// process on one GPU.  The scheduling policy (queue, dispatcher thread, slots, resident
// plans under the HBM budget, statistics) is ServerCore in lgf_server_core.h; this file is
// its executor on the device and the C ABI of lgf.h.
//
// Executor: each stream slot is a non-blocking HIP stream; a request's solve runs on its
// slot's stream after an event recorded on the submitter's stream at submit time, between
// two timing events, and is retired when the second has fired.  Plans are lgf_plan_create
// plans of the server's (n, p, levels, precision); kernel spectra live in the library-wide
// cache keyed by (n, p, level, precision), so every plan shares them.
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_internal.h"
#include "lgf_server_core.h"

using namespace lgfdev;

namespace {

struct HipExec {
    using Plan = lgf_plan_t;
    struct Job {
        const void* f = nullptr;
        void* u = nullptr;
        // recorded on the submitter's stream at submit time: the slot stream waits for it,
        // so the solve reads f (and overwrites u) only after the work the caller queued
        // before the submit
        hipEvent_t ev_ready = nullptr;
        hipEvent_t ev_start = nullptr, ev_end = nullptr;
    };

    lgf_server_config cfg{};
    int device = 0;
    int spectra_mode = 0;  // kernel spectra of the server's plans: the process-wide mode at creation
    std::vector<hipStream_t> slots;
    std::mutex pool_mu;               // events are taken by submitting threads and the dispatcher
    std::vector<hipEvent_t> pool;     // timing events
    std::vector<hipEvent_t> ready;    // submit-time events (no timing)

    ~HipExec() {
        for (auto s : slots) hipStreamSynchronize(s);
        for (auto e : pool) hipEventDestroy(e);
        for (auto e : ready) hipEventDestroy(e);
        for (auto s : slots) hipStreamDestroy(s);
    }

    hipEvent_t take(std::vector<hipEvent_t>& from, unsigned flags) {
        {
            std::lock_guard<std::mutex> lk(pool_mu);
            if (!from.empty()) {
                hipEvent_t e = from.back();
                from.pop_back();
                return e;
            }
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, flags) != hipSuccess) return nullptr;
        return e;
    }
    void give(std::vector<hipEvent_t>& to, hipEvent_t& e) {
        if (!e) return;
        std::lock_guard<std::mutex> lk(pool_mu);
        to.push_back(e);
        e = nullptr;
    }

    void thread_init() {
        hipSetDevice(device);
        spectra_set_thread_mode(spectra_mode);  // the plans the dispatcher creates
    }

    lgf_status estimate(const std::vector<int32_t>& layout, int64_t* bytes, std::string* err) {
        const lgf_status st = plan_estimate(layout.data(), (int64_t)layout.size() / 3, cfg.n, cfg.p, cfg.levels,
                                            (lgf_precision)cfg.precision, bytes);
        if (st != LGF_OK) *err = lgf_last_error();
        return st;
    }

    int64_t shared_bytes() { return spectra_bytes_total(); }

    lgf_status create(const std::vector<int32_t>& layout, int slot, Plan* out, int64_t* bytes, std::string* err) {
        lgf_status st = lgf_plan_create(layout.data(), (int64_t)layout.size() / 3, cfg.n, cfg.p, cfg.levels,
                                        (lgf_precision)cfg.precision, slots[slot], out);
        if (st != LGF_OK) {
            *err = lgf_last_error();
            return st;
        }
        lgf_plan_info info;
        lgf_plan_query(*out, &info);
        *bytes = info.workspace_bytes;
        return LGF_OK;
    }

    void destroy(Plan plan) { lgf_plan_destroy(plan); }

    lgf_status start(Job& job, Plan plan, int slot, std::string* err) {
        job.ev_start = take(pool, hipEventDefault);
        job.ev_end = take(pool, hipEventDefault);
        if (!job.ev_start || !job.ev_end) {
            *err = "event creation failed";
            return LGF_ERR_DEVICE;
        }
        hipStream_t s = slots[slot];
        // the solve follows everything the submitter had queued on its stream before the submit
        if (hipStreamWaitEvent(s, job.ev_ready, 0) != hipSuccess) {
            *err = "stream wait on the submit event failed";
            return LGF_ERR_DEVICE;
        }
        hipEventRecord(job.ev_start, s);
        const lgf_status st = lgf_solve(plan, job.f, job.u, s);
        hipEventRecord(job.ev_end, s);
        if (st != LGF_OK) *err = lgf_last_error();
        return st;
    }

    int query(Job& job, double* device_ms, std::string* err) {
        const hipError_t q = hipEventQuery(job.ev_end);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) {
            *err = std::string("solve failed: ") + hipGetErrorString(q);
            return -1;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, job.ev_start, job.ev_end) == hipSuccess) *device_ms = ms;
        return 1;
    }

    void release(Job& job) {
        give(ready, job.ev_ready);
        give(pool, job.ev_start);
        give(pool, job.ev_end);
    }
};

using Core = ServerCore<HipExec>;

}  // namespace

struct lgf_server_s {
    HipExec ex;                  // destroyed after the core: the core's plans and events first
    std::unique_ptr<Core> core;  // its destructor drains the queue and joins the dispatcher
    ~lgf_server_s() { core.reset(); }
};

extern "C" {

lgf_status lgf_server_create(const lgf_server_config* cfg, lgf_server_t* out) {
    if (!out || !cfg) {
        set_last_error("NULL argument to lgf_server_create");
        return LGF_ERR_ARG;
    }
    *out = nullptr;
    if (!block_edge_ok(cfg->n)) {
        set_last_error("n must be 4, 6, 8, 12 or 16");
        return LGF_ERR_ARG;
    }
    if (!nodes_ok(cfg->n, cfg->p) ||
        (cfg->precision != LGF_F64 && cfg->precision != LGF_F32) ||
        cfg->max_slots < 1 || cfg->max_slots > 16 || cfg->budget_bytes < 0 || cfg->max_queue < 0) {
        set_last_error("lgf_server_create: p in [2, 10] (or n + 1 with n = 12, 16), precision, max_slots in [1, 16], budget >= 0");
        return LGF_ERR_ARG;
    }
    auto S = std::make_unique<lgf_server_s>();
    S->ex.cfg = *cfg;
    S->ex.spectra_mode = spectra_mode();
    if (hipGetDevice(&S->ex.device) != hipSuccess) {
        set_last_error("no HIP device");
        return LGF_ERR_DEVICE;
    }
    for (int k = 0; k < cfg->max_slots; ++k) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            set_last_error("stream creation failed");
            return LGF_ERR_DEVICE;
        }
        S->ex.slots.push_back(s);
    }
    Core::Config cc;
    cc.max_slots = cfg->max_slots;
    cc.budget_bytes = cfg->budget_bytes;
    cc.max_queue = cfg->max_queue;
    cc.points_per_block = (int64_t)cfg->n * cfg->n * cfg->n;
    S->core = std::make_unique<Core>(S->ex, cc);
    *out = S.release();
    return LGF_OK;
}

lgf_status lgf_server_submit(lgf_server_t S, const int32_t* block_ijk, int64_t nblocks, const void* f, void* u,
                             void* hip_stream, int64_t* ticket) {
    if (!S || !block_ijk || !f || !u || !ticket || nblocks < 1) {
        set_last_error("bad arguments to lgf_server_submit");
        return LGF_ERR_ARG;
    }
    HipExec::Job job;
    job.f = f;
    job.u = u;
    job.ev_ready = S->ex.take(S->ex.ready, hipEventDisableTiming);
    if (!job.ev_ready) {
        set_last_error("event creation failed in lgf_server_submit");
        return LGF_ERR_DEVICE;
    }
    if (hipEventRecord(job.ev_ready, (hipStream_t)hip_stream) != hipSuccess) {
        S->ex.release(job);
        set_last_error("lgf_server_submit: recording on the caller's stream failed");
        return LGF_ERR_DEVICE;
    }
    std::string err;
    const lgf_status st =
        S->core->submit(std::vector<int32_t>(block_ijk, block_ijk + 3 * nblocks), nblocks, job, ticket, &err);
    if (st != LGF_OK) {
        S->ex.release(job);  // not taken by the core
        set_last_error(err);
    }
    return st;
}

static void fill_result(const Core::Result& r, lgf_request_result* res) {
    if (r.status != LGF_OK) set_last_error(r.error);
    if (!res) return;
    std::memset(res, 0, sizeof(*res));
    res->status = r.status;
    res->latency_ms = r.latency_ms;
    res->queue_ms = r.queue_ms;
    res->device_ms = r.device_ms;
    res->nblocks = r.nblocks;
}

lgf_status lgf_server_poll(lgf_server_t S, int64_t ticket, int32_t* done, lgf_request_result* res) {
    if (!S || !done) {
        set_last_error("bad arguments to lgf_server_poll");
        return LGF_ERR_ARG;
    }
    bool d = false;
    Core::Result r;
    if (S->core->poll(ticket, &d, &r) != LGF_OK) {
        set_last_error("unknown ticket");
        return LGF_ERR_ARG;
    }
    *done = d ? 1 : 0;
    if (d) fill_result(r, res);
    return LGF_OK;
}

lgf_status lgf_server_wait(lgf_server_t S, int64_t ticket, lgf_request_result* res) {
    if (!S) {
        set_last_error("NULL server");
        return LGF_ERR_ARG;
    }
    Core::Result r;
    if (S->core->wait(ticket, &r) != LGF_OK) {
        set_last_error("unknown ticket");
        return LGF_ERR_ARG;
    }
    fill_result(r, res);
    return LGF_OK;
}

lgf_status lgf_server_stats(lgf_server_t S, lgf_server_stats_t* out) {
    if (!S || !out) {
        set_last_error("bad arguments to lgf_server_stats");
        return LGF_ERR_ARG;
    }
    const Core::Stats s = S->core->stats();
    std::memset(out, 0, sizeof(*out));
    out->completed = s.completed;
    out->failed = s.failed;
    out->queued = s.queued;
    out->points = s.points;
    out->plans_created = s.plans_created;
    out->plans_evicted = s.plans_evicted;
    out->plan_bytes = s.plan_bytes;
    out->spectra_bytes = spectra_bytes_total();
    out->latency_p50_ms = s.p50_ms;
    out->latency_p99_ms = s.p99_ms;
    out->latency_max_ms = s.max_ms;
    out->points_per_s = s.points_per_s;
    return LGF_OK;
}

lgf_status lgf_server_reset_stats(lgf_server_t S) {
    if (!S) {
        set_last_error("NULL server");
        return LGF_ERR_ARG;
    }
    S->core->reset_stats();
    return LGF_OK;
}

lgf_status lgf_server_destroy(lgf_server_t S) {
    delete S;  // drains the queue, joins the dispatcher, releases plans, events and streams
    return LGF_OK;
}

}  // extern "C"
