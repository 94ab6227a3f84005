// Scheduling core of the request server, free of device calls: the request queue and its
// tickets, the dispatcher thread, stream-slot assignment, the cache of resident plans with
// least-recently-used eviction under an HBM budget, and the latency statistics.  Each
// request is one solve u = G * f (Sec. 3.1); how a plan is built and a solve is issued and
// observed is the executor's business (the template parameter), so the policy here runs the
// same against the GPU and against a host mock in the tests.
//
// Exec provides (all called from the dispatcher thread unless noted):
//   typename Exec::Plan, typename Exec::Job   handles; Job is the per-request device state
//   void thread_init()                         once, at the start of the dispatcher thread
//   lgf_status estimate(const std::vector<int32_t>& layout, int64_t* bytes, std::string* err)
//   int64_t shared_bytes()                     resident bytes every plan shares (kernel spectra)
//   lgf_status create(const std::vector<int32_t>& layout, int slot, Plan* out, int64_t* bytes,
//                     std::string* err)
//   void destroy(Plan plan)
//   lgf_status start(Job& job, Plan plan, int slot, std::string* err)   issue the solve
//   int query(Job& job, double* device_ms, std::string* err)  0 running, 1 done, -1 failed
//   void release(Job& job)                     the request is finished (any thread, under no lock
//                                              of the core); give back its resources
//
// Policy.  Requests are admitted in arrival order: the head of the queue waits until a slot
// is free and its plan is resident or fits the budget (idle resident plans are evicted, least
// recently used first, to make room); a request whose plan cannot fit even alone fails with
// LGF_ERR_BUDGET and the queue moves on.  A plan serves one request at a time; a second
// concurrent request of the same layout gets a second plan if the budget allows, else waits.
#ifndef LGF_SERVER_CORE_H_
#define LGF_SERVER_CORE_H_

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lgf.h"

namespace lgfdev {

template <class Exec>
class ServerCore {
public:
    using Plan = typename Exec::Plan;
    using Job = typename Exec::Job;
    using Clock = std::chrono::steady_clock;

    struct Config {
        int max_slots = 1;
        int64_t budget_bytes = 0;      // 0: unlimited
        int64_t max_queue = 0;         // 0: unlimited
        int64_t points_per_block = 0;  // for the points statistic
    };

    struct Result {
        lgf_status status = LGF_OK;
        std::string error;
        double latency_ms = 0, queue_ms = 0, device_ms = 0;
        int64_t nblocks = 0;
    };

    struct Stats {
        int64_t completed = 0, failed = 0, queued = 0, points = 0;
        int64_t plans_created = 0, plans_evicted = 0, plan_bytes = 0;
        double p50_ms = 0, p99_ms = 0, max_ms = 0, points_per_s = 0;
    };

    ServerCore(Exec& ex, const Config& cfg) : ex_(ex), cfg_(cfg), slot_busy_(cfg.max_slots, false) {
        worker_ = std::thread([this] { dispatch(); });
    }

    // Drains the queue (every submitted request still runs), then destroys the plans.
    ~ServerCore() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (worker_.joinable()) worker_.join();
        for (auto& cp : plans_) ex_.destroy(cp->plan);
        for (auto& kv : tickets_)
            if (!kv.second->released) ex_.release(kv.second->job);
    }

    // Queue one request (any thread).  On failure the job is not taken: the caller keeps it.
    // Errors: LGF_ERR_BUSY (queue full), LGF_ERR_ARG (shutting down).
    lgf_status submit(std::vector<int32_t> layout, int64_t nblocks, Job job, int64_t* ticket, std::string* err) {
        auto r = std::make_shared<Req>();
        r->key.assign(reinterpret_cast<const char*>(layout.data()), layout.size() * sizeof(int32_t));
        r->layout = std::move(layout);
        r->nblocks = nblocks;
        r->t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stop_) {
                *err = "server is shutting down";
                return LGF_ERR_ARG;
            }
            if (cfg_.max_queue > 0 && (int64_t)queue_.size() >= cfg_.max_queue) {
                *err = "request queue is full";
                return LGF_ERR_BUSY;
            }
            r->job = std::move(job);
            r->ticket = next_ticket_++;
            queue_.push_back(r);
            tickets_[r->ticket] = r;
            if (!any_submit_) {
                any_submit_ = true;
                t_first_submit_ = r->t_submit;
            }
            *ticket = r->ticket;
        }
        cv_work_.notify_one();
        return LGF_OK;
    }

    // done = false while the request runs; once done the ticket is released.
    // Errors: LGF_ERR_ARG (unknown or released ticket).
    lgf_status poll(int64_t ticket, bool* done, Result* res) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return LGF_ERR_ARG;
        *done = it->second->done;
        if (*done) {
            *res = result_of(*it->second);
            tickets_.erase(it);
        }
        return LGF_OK;
    }

    lgf_status wait(int64_t ticket, Result* res) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = tickets_.find(ticket);
        if (it == tickets_.end()) return LGF_ERR_ARG;
        std::shared_ptr<Req> r = it->second;
        cv_done_.wait(lk, [&] { return r->done; });
        *res = result_of(*r);
        tickets_.erase(ticket);
        return LGF_OK;
    }

    Stats stats() {
        std::lock_guard<std::mutex> lk(mu_);
        Stats s;
        s.completed = completed_;
        s.failed = failed_;
        s.queued = (int64_t)queue_.size();
        s.points = points_;
        s.plans_created = plans_created_;
        s.plans_evicted = plans_evicted_;
        s.plan_bytes = plan_bytes_pub_;
        if (!latencies_ms_.empty()) {
            std::vector<double> v = latencies_ms_;
            std::sort(v.begin(), v.end());
            auto pct = [&](double q) {
                const double pos = q * (double)(v.size() - 1);
                const size_t i = (size_t)pos;
                const double fr = pos - (double)i;
                return i + 1 < v.size() ? v[i] * (1.0 - fr) + v[i + 1] * fr : v[i];
            };
            s.p50_ms = pct(0.50);
            s.p99_ms = pct(0.99);
            s.max_ms = v.back();
            const double span = ms(t_first_submit_, t_last_done_);
            s.points_per_s = span > 0 ? (double)points_ / (span * 1e-3) : 0.0;
        }
        return s;
    }

    void reset_stats() {
        std::lock_guard<std::mutex> lk(mu_);
        latencies_ms_.clear();
        completed_ = failed_ = points_ = 0;
        any_submit_ = false;
    }

private:
    struct Resident {
        std::string key;
        Plan plan{};
        int64_t bytes = 0;
        bool busy = false;
        uint64_t last_use = 0;
    };

    struct Req {
        int64_t ticket = 0;
        std::vector<int32_t> layout;
        std::string key;
        int64_t nblocks = 0;
        Job job{};
        Clock::time_point t_submit, t_start, t_done;
        bool started = false;
        lgf_status status = LGF_OK;
        std::string error;
        bool done = false, released = false;
        int slot = -1;
        Resident* cp = nullptr;
        double device_ms = 0.0;
    };

    static double ms(Clock::time_point a, Clock::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    }

    static Result result_of(const Req& r) {
        Result res;
        res.status = r.status;
        res.error = r.error;
        res.latency_ms = ms(r.t_submit, r.t_done);
        res.queue_ms = r.started ? ms(r.t_submit, r.t_start) : 0.0;
        res.device_ms = r.device_ms;
        res.nblocks = r.nblocks;
        return res;
    }

    void finish(const std::shared_ptr<Req>& r, lgf_status st, const std::string& err) {
        ex_.release(r->job);
        std::lock_guard<std::mutex> lk(mu_);
        r->released = true;
        r->status = st;
        r->error = err;
        r->done = true;
        r->t_done = Clock::now();
        if (st == LGF_OK) {
            ++completed_;
            points_ += r->nblocks * cfg_.points_per_block;
            latencies_ms_.push_back(ms(r->t_submit, r->t_done));
            t_last_done_ = r->t_done;
        } else {
            ++failed_;
        }
        plan_bytes_pub_ = plan_bytes_;
        cv_done_.notify_all();
    }

    // Retire the running requests whose solves have ended.
    void retire() {
        for (size_t i = 0; i < inflight_.size();) {
            auto r = inflight_[i];
            std::string err;
            const int q = ex_.query(r->job, &r->device_ms, &err);
            if (q == 0) {
                ++i;
                continue;
            }
            r->cp->busy = false;
            r->cp->last_use = ++use_clock_;
            slot_busy_[r->slot] = false;
            inflight_[i] = inflight_.back();
            inflight_.pop_back();
            finish(r, q > 0 ? LGF_OK : LGF_ERR_DEVICE, q > 0 ? std::string() : err);
        }
    }

    int64_t resident_bytes() { return plan_bytes_ + ex_.shared_bytes(); }

    void count(int64_t& c) {
        std::lock_guard<std::mutex> lk(mu_);
        ++c;
        plan_bytes_pub_ = plan_bytes_;
    }

    // Start the request at the head of the queue.  Returns true if it started or failed
    // (the queue moves on), false if it has to wait.
    bool try_admit(const std::shared_ptr<Req>& r) {
        int slot = -1;
        for (size_t k = 0; k < slot_busy_.size(); ++k)
            if (!slot_busy_[k]) {
                slot = (int)k;
                break;
            }
        if (slot < 0) return false;
        Resident* cp = nullptr;
        for (auto& c : plans_)
            if (!c->busy && c->key == r->key) {
                cp = c.get();
                break;
            }
        if (!cp) {
            int64_t est = 0;
            std::string err;
            lgf_status st = ex_.estimate(r->layout, &est, &err);
            if (st != LGF_OK) {
                finish(r, st, err);
                return true;
            }
            const int64_t budget = cfg_.budget_bytes;
            if (budget > 0 && est + ex_.shared_bytes() > budget) {
                finish(r, LGF_ERR_BUDGET, "request exceeds the server's HBM budget on its own");
                return true;
            }
            // evict idle plans, least recently used first, until the new one fits
            while (budget > 0 && resident_bytes() + est > budget) {
                auto victim = plans_.end();
                for (auto it = plans_.begin(); it != plans_.end(); ++it)
                    if (!(*it)->busy && (victim == plans_.end() || (*it)->last_use < (*victim)->last_use))
                        victim = it;
                if (victim == plans_.end()) break;
                plan_bytes_ -= (*victim)->bytes;
                ex_.destroy((*victim)->plan);
                plans_.erase(victim);
                count(plans_evicted_);
            }
            if (budget > 0 && resident_bytes() + est > budget) return false;  // wait for running work
            Plan pl{};
            int64_t bytes = 0;
            st = ex_.create(r->layout, slot, &pl, &bytes, &err);
            if (st != LGF_OK) {
                finish(r, st, err);
                return true;
            }
            auto c = std::make_unique<Resident>();
            c->key = r->key;
            c->plan = pl;
            c->bytes = bytes;
            cp = c.get();
            plans_.push_back(std::move(c));
            plan_bytes_ += bytes;
            count(plans_created_);
        }
        r->t_start = Clock::now();
        r->started = true;
        std::string err;
        const lgf_status st = ex_.start(r->job, cp->plan, slot, &err);
        if (st != LGF_OK) {
            finish(r, st, err);
            return true;
        }
        cp->busy = true;
        r->cp = cp;
        r->slot = slot;
        slot_busy_[slot] = true;
        inflight_.push_back(r);
        return true;
    }

    void dispatch() {
        ex_.thread_init();
        for (;;) {
            retire();
            std::shared_ptr<Req> head;
            {
                std::unique_lock<std::mutex> lk(mu_);
                if (queue_.empty()) {
                    if (stop_ && inflight_.empty()) return;
                    if (inflight_.empty()) {
                        cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
                        continue;
                    }
                } else {
                    head = queue_.front();
                }
            }
            bool advanced = false;
            if (head) {
                advanced = try_admit(head);
                if (advanced) {
                    std::lock_guard<std::mutex> lk(mu_);
                    queue_.pop_front();
                }
            }
            // nothing to start: poll the running requests
            if (!advanced && !inflight_.empty()) std::this_thread::yield();
        }
    }

    Exec& ex_;
    const Config cfg_;

    std::mutex mu_;
    std::condition_variable cv_work_;  // new request or shutdown
    std::condition_variable cv_done_;  // a request finished
    std::deque<std::shared_ptr<Req>> queue_;
    std::map<int64_t, std::shared_ptr<Req>> tickets_;
    int64_t next_ticket_ = 1;
    bool stop_ = false;

    // dispatcher-owned
    std::vector<bool> slot_busy_;
    std::vector<std::shared_ptr<Req>> inflight_;
    std::list<std::unique_ptr<Resident>> plans_;
    int64_t plan_bytes_ = 0;
    uint64_t use_clock_ = 0;

    // statistics (under mu_)
    std::vector<double> latencies_ms_;
    int64_t completed_ = 0, failed_ = 0, points_ = 0, plans_created_ = 0, plans_evicted_ = 0;
    int64_t plan_bytes_pub_ = 0;  // plan_bytes_ as of the last change, for stats()
    Clock::time_point t_first_submit_, t_last_done_;
    bool any_submit_ = false;

    std::thread worker_;  // started by the constructor, joined by the destructor
};

}  // namespace lgfdev

#endif  // LGF_SERVER_CORE_H_
