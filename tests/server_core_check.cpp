// Host checks of the request server's scheduling core (ServerCore, lgf_server_core.h) with a
// mock executor instead of the GPU: admission order, stream-slot and plan exclusivity, the
// HBM budget with least-recently-used eviction, refusal of requests too large for the
// budget, waiting for running work, the queue limit, failure injection at every executor
// step, ticket handling, statistics and shutdown.  Built with the address and undefined-
// behaviour sanitizers, and separately with the thread sanitizer, by tests/test_host_sanitized.py.
// Prints one line per scenario; exits non-zero on the first failed check.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "lgf_server_core.h"

namespace {

int g_fail = 0;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "check failed: %s (%s:%d)\n", #cond, __FILE__, __LINE__); \
            ++g_fail;                                                                 \
        }                                                                             \
    } while (0)

// Layout markers: the first coordinate of a layout selects an injected failure.
constexpr int kBadEstimate = -7, kBadCreate = -8;

struct MockExec {
    using Plan = int;
    struct Job {
        int id = -1;
        int run_polls = 0;        // polls that report "running" once the gate is open
        bool fail_start = false;  // start() fails
        bool fail_run = false;    // the solve fails (query -1)
        int plan = -1, slot = -1; // set by start()
    };

    explicit MockExec(int slots, int64_t budget, int64_t per_block = 1000, int64_t shared = 500)
        : budget(budget), per_block(per_block), shared(shared), slot_busy(slots, false) {}

    // configuration
    int64_t budget, per_block, shared;
    std::atomic<bool> gate{true};  // while false every started solve stays running

    // dispatcher-side state
    struct Live {
        int64_t bytes = 0;
        bool busy = false;
    };
    std::map<int, Live> live;
    int64_t live_bytes = 0, peak_bytes = 0;
    int next_plan = 1, created = 0;
    std::vector<int> destroyed, started;
    std::vector<bool> slot_busy;
    std::thread::id dispatcher;
    bool inited = false;

    // released jobs (any thread)
    std::mutex mu;
    std::multiset<int> released;

    void on_dispatcher() { CHECK(std::this_thread::get_id() == dispatcher); }

    void thread_init() {
        dispatcher = std::this_thread::get_id();
        inited = true;
    }

    lgf_status estimate(const std::vector<int32_t>& layout, int64_t* bytes, std::string* err) {
        on_dispatcher();
        if (layout[0] == kBadEstimate) {
            *err = "injected layout error";
            return LGF_ERR_LAYOUT;
        }
        *bytes = (int64_t)layout.size() / 3 * per_block;
        return LGF_OK;
    }

    int64_t shared_bytes() { return shared; }

    lgf_status create(const std::vector<int32_t>& layout, int slot, Plan* out, int64_t* bytes, std::string* err) {
        on_dispatcher();
        CHECK(slot >= 0 && slot < (int)slot_busy.size() && !slot_busy[slot]);
        if (layout[0] == kBadCreate) {
            *err = "injected allocation failure";
            return LGF_ERR_OOM;
        }
        const int64_t b = (int64_t)layout.size() / 3 * per_block;
        CHECK(budget == 0 || live_bytes + shared + b <= budget);  // the budget holds at every creation
        *out = next_plan++;
        *bytes = b;
        live[*out] = Live{b, false};
        live_bytes += b;
        peak_bytes = std::max(peak_bytes, live_bytes);
        ++created;
        return LGF_OK;
    }

    void destroy(Plan p) {
        auto it = live.find(p);
        CHECK(it != live.end());
        if (it == live.end()) return;
        CHECK(!it->second.busy);  // never a plan that is serving a request
        live_bytes -= it->second.bytes;
        live.erase(it);
        destroyed.push_back(p);
    }

    lgf_status start(Job& job, Plan p, int slot, std::string* err) {
        on_dispatcher();
        CHECK(live.count(p) == 1 && !live[p].busy);            // one request per plan
        CHECK(slot >= 0 && slot < (int)slot_busy.size() && !slot_busy[slot]);  // one per slot
        if (job.fail_start) {
            *err = "injected launch failure";
            return LGF_ERR_DEVICE;
        }
        live[p].busy = true;
        slot_busy[slot] = true;
        job.plan = p;
        job.slot = slot;
        started.push_back(job.id);
        return LGF_OK;
    }

    int query(Job& job, double* device_ms, std::string* err) {
        on_dispatcher();
        if (!gate.load()) return 0;
        if (job.run_polls > 0) {
            --job.run_polls;
            return 0;
        }
        live[job.plan].busy = false;
        slot_busy[job.slot] = false;
        *device_ms = 0.25;
        if (job.fail_run) {
            *err = "injected device fault";
            return -1;
        }
        return 1;
    }

    void release(Job& job) {
        std::lock_guard<std::mutex> lk(mu);
        released.insert(job.id);
    }
};

using Core = lgfdev::ServerCore<MockExec>;

std::vector<int32_t> layout(int tag, int nblocks) {
    std::vector<int32_t> v;
    for (int b = 0; b < nblocks; ++b) {
        v.push_back(tag);
        v.push_back(b);
        v.push_back(0);
    }
    return v;
}

Core::Config config(int slots, int64_t budget, int64_t max_queue = 0) {
    Core::Config c;
    c.max_slots = slots;
    c.budget_bytes = budget;
    c.max_queue = max_queue;
    c.points_per_block = 4096;
    return c;
}

int64_t submit(Core& core, int tag, int nblocks, MockExec::Job job, lgf_status want = LGF_OK) {
    int64_t t = -1;
    std::string err;
    const lgf_status st = core.submit(layout(tag, nblocks), nblocks, job, &t, &err);
    CHECK(st == want);
    return st == LGF_OK ? t : -1;
}

Core::Result wait(Core& core, int64_t t) {
    Core::Result r;
    CHECK(core.wait(t, &r) == LGF_OK);
    return r;
}

MockExec::Job job(int id, int polls = 0) {
    MockExec::Job j;
    j.id = id;
    j.run_polls = polls;
    return j;
}

void scenario_fifo_and_reuse() {
    MockExec ex(2, 0);
    std::vector<int64_t> tickets;
    {
        Core core(ex, config(2, 0));
        for (int i = 0; i < 40; ++i) tickets.push_back(submit(core, i % 5, 3 + i % 5, job(i, i % 3)));
        int64_t pts = 0;
        for (int i = 0; i < 40; ++i) {
            const Core::Result r = wait(core, tickets[i]);
            CHECK(r.status == LGF_OK && r.nblocks == 3 + i % 5);
            CHECK(r.latency_ms >= r.queue_ms && r.queue_ms >= 0.0 && r.device_ms == 0.25);
            pts += (3 + i % 5) * 4096;
        }
        const Core::Stats s = core.stats();
        CHECK(s.completed == 40 && s.failed == 0 && s.queued == 0 && s.points == pts);
        CHECK(s.plans_created <= 10 && s.plans_evicted == 0);  // at most two instances per layout
        CHECK(0 <= s.p50_ms && s.p50_ms <= s.p99_ms && s.p99_ms <= s.max_ms);
        Core::Result r;
        bool done = false;
        CHECK(core.poll(tickets[0], &done, &r) == LGF_ERR_ARG);  // released by the wait
        CHECK(core.poll(987654, &done, &r) == LGF_ERR_ARG);
    }
    CHECK(ex.inited);
    for (int i = 0; i < 40; ++i) CHECK(ex.started[i] == i);  // admitted in arrival order
    CHECK(ex.released.size() == 40 && std::set<int>(ex.released.begin(), ex.released.end()).size() == 40);
    CHECK((int)ex.destroyed.size() == ex.created && ex.live.empty());  // no plan outlives the server
    std::printf("ok fifo, plan reuse, statistics, tickets\n");
}

void scenario_lru_eviction() {
    // budget for the shared bytes and two plans of 4 blocks; one slot, so each request
    // finishes before the next is admitted
    MockExec ex(1, 500 + 2 * 4000);
    {
        Core core(ex, config(1, 500 + 2 * 4000));
        const int order[] = {1, 2, 1, 3, 1, 2};
        int id = 0;
        for (int tag : order) CHECK(wait(core, submit(core, tag, 4, job(id++))).status == LGF_OK);
        const Core::Stats s = core.stats();
        // A, B resident; C evicts B (A was used more recently); A reused; B evicts C
        CHECK(s.plans_created == 4 && s.plans_evicted == 2);
        CHECK(ex.destroyed.size() >= 2 && ex.destroyed[0] == 2 && ex.destroyed[1] == 3);
        CHECK(s.plan_bytes == 2 * 4000);
    }
    CHECK(ex.peak_bytes <= 2 * 4000);
    std::printf("ok least-recently-used eviction under the budget\n");
}

void scenario_budget_refusal_and_waiting() {
    MockExec ex(2, 500 + 6000);
    {
        Core core(ex, config(2, 500 + 6000));
        // too large on its own: refused, the queue moves on
        const int64_t big = submit(core, 1, 7, job(0));
        const int64_t ok = submit(core, 2, 6, job(1));
        CHECK(wait(core, big).status == LGF_ERR_BUDGET);
        CHECK(wait(core, ok).status == LGF_OK);
        // two layouts that cannot be resident together: the second waits for the first to end
        // (a running plan is never evicted), although a slot is free
        ex.gate = false;
        const int64_t a = submit(core, 3, 5, job(2));
        const int64_t b = submit(core, 4, 5, job(3));
        std::this_thread::sleep_for(std::chrono::milliseconds(50));
        Core::Result r;
        bool done = true;
        CHECK(core.poll(b, &done, &r) == LGF_OK && !done);
        CHECK(core.stats().queued == 1);
        ex.gate = true;
        CHECK(wait(core, a).status == LGF_OK);
        CHECK(wait(core, b).status == LGF_OK);
        const Core::Stats s = core.stats();
        CHECK(s.completed == 3 && s.failed == 1);
    }
    CHECK(ex.peak_bytes <= 6000);
    std::printf("ok refusal of oversize requests, waiting for running work\n");
}

void scenario_queue_limit() {
    MockExec ex(1, 0);
    {
        Core core(ex, config(1, 0, 3));
        ex.gate = false;
        std::vector<int64_t> accepted;
        int busy = 0;
        for (int i = 0; i < 8; ++i) {
            int64_t t = -1;
            std::string err;
            const lgf_status st = core.submit(layout(1, 2), 2, job(i), &t, &err);
            if (st == LGF_OK)
                accepted.push_back(t);
            else {
                CHECK(st == LGF_ERR_BUSY && err == "request queue is full");
                ++busy;
            }
        }
        CHECK(busy >= 4 && accepted.size() <= 4 && accepted.size() >= 3);
        ex.gate = true;
        for (int64_t t : accepted) CHECK(wait(core, t).status == LGF_OK);
        CHECK(core.stats().completed == (int64_t)accepted.size());
    }
    CHECK(ex.released.size() == ex.started.size());  // refused jobs were never taken
    std::printf("ok queue limit\n");
}

void scenario_failures() {
    MockExec ex(2, 0);
    {
        Core core(ex, config(2, 0));
        MockExec::Job fs = job(2), fr = job(3);
        fs.fail_start = true;
        fr.fail_run = true;
        const int64_t t0 = submit(core, kBadEstimate, 2, job(0));
        const int64_t t1 = submit(core, kBadCreate, 2, job(1));
        const int64_t t2 = submit(core, 5, 2, fs);
        const int64_t t3 = submit(core, 6, 2, fr);
        const int64_t t4 = submit(core, 6, 2, job(4));  // reuses the plan the failed solve left idle
        const int64_t t5 = submit(core, 5, 2, job(5));
        Core::Result r = wait(core, t0);
        CHECK(r.status == LGF_ERR_LAYOUT && r.error == "injected layout error");
        CHECK(wait(core, t1).status == LGF_ERR_OOM);
        CHECK(wait(core, t2).status == LGF_ERR_DEVICE);
        r = wait(core, t3);
        CHECK(r.status == LGF_ERR_DEVICE && r.error == "injected device fault");
        CHECK(wait(core, t4).status == LGF_OK);
        CHECK(wait(core, t5).status == LGF_OK);
        const Core::Stats s = core.stats();
        CHECK(s.completed == 2 && s.failed == 4);
        CHECK(s.plans_created <= 3);
    }
    CHECK(ex.released.size() == 6);
    std::printf("ok failures at estimate, creation, launch and on the device\n");
}

void scenario_concurrent_clients() {
    MockExec ex(4, 500 + 5 * 8000);
    std::atomic<int> ok{0}, refused{0};
    constexpr int kThreads = 8, kPer = 150;
    {
        Core core(ex, config(4, 500 + 5 * 8000));
        std::vector<std::thread> th;
        for (int t = 0; t < kThreads; ++t)
            th.emplace_back([&, t] {
                std::mt19937 rng(1234 + t);
                std::vector<std::pair<int64_t, int>> mine;
                for (int i = 0; i < kPer; ++i) {
                    const int tag = (int)(rng() % 10), nb = 1 + tag % 8;
                    MockExec::Job j = job(t * kPer + i, (int)(rng() % 4));
                    int64_t tk = -1;
                    std::string err;
                    if (core.submit(layout(tag, nb), nb, j, &tk, &err) == LGF_OK) mine.push_back({tk, nb});
                    if (rng() % 5 == 0 && !mine.empty()) {  // some clients poll, others wait
                        Core::Result r;
                        bool done = false;
                        if (core.poll(mine.front().first, &done, &r) == LGF_OK && done) {
                            (r.status == LGF_OK ? ok : refused)++;
                            mine.erase(mine.begin());
                        }
                    }
                }
                for (auto& m : mine) {
                    Core::Result r;
                    CHECK(core.wait(m.first, &r) == LGF_OK);
                    CHECK(r.nblocks == m.second);
                    (r.status == LGF_OK ? ok : refused)++;
                }
            });
        for (auto& x : th) x.join();
        const Core::Stats s = core.stats();
        CHECK(s.completed == ok.load() && s.failed == refused.load() && s.queued == 0);
    }
    CHECK(ok.load() + refused.load() == kThreads * kPer && refused.load() == 0);
    CHECK(ex.peak_bytes <= 5 * 8000 && ex.live.empty());
    CHECK((int)ex.released.size() == kThreads * kPer);
    std::printf("ok %d concurrent clients, %d requests\n", kThreads, kThreads * kPer);
}

void scenario_shutdown_drains() {
    MockExec ex(2, 500 + 3 * 3000);
    {
        Core core(ex, config(2, 500 + 3 * 3000));
        for (int i = 0; i < 60; ++i) submit(core, i % 7, 3, job(i, i % 2));
        // destroyed with every request still queued or running, no ticket waited on
    }
    CHECK(ex.started.size() == 60 && ex.released.size() == 60);
    CHECK((int)ex.destroyed.size() == ex.created && ex.live.empty());
    std::printf("ok shutdown drains the queue\n");
}

}  // namespace

int main() {
    scenario_fifo_and_reuse();
    scenario_lru_eviction();
    scenario_budget_refusal_and_waiting();
    scenario_queue_limit();
    scenario_failures();
    scenario_concurrent_clients();
    scenario_shutdown_drains();
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("all server-core checks passed\n");
    return 0;
}
