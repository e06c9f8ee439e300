// rr_server_core.h -- the host side of the serving loop (continuous
// batching), independent of the device.
//
// ServerCore owns the request queue, the slots, the completions and the
// worker thread; it decides what each tick admits and what it returns or
// retries.  The device work of a tick (staging the admitted queries, running
// the search kernels over the resident slots, reading back states and
// results) is done by a Dev object:
//
//   bool stage(int32_t k, int32_t slot, const ServerRequest &r)
//       admitted request k of this tick goes to `slot` (host-side staging);
//   bool tick(int32_t admitted, const int32_t *active, int32_t nwork, std::string &err)
//       one tick over the resident slots active[0, nwork) (the first
//       `admitted` staged requests are new); false with a message on failure;
//   SlotOutcome outcome(int32_t slot) const
//       after a tick: has the slot's search finished, and its statistics;
//   bool shared_overflow() const
//       after a tick: a capacity shared by the tick's queries ran out;
//   bool result(int32_t slot, ServerFinished &f, std::string &err) const
//       after a tick: the finished slot's ids and distances.
//
// rr_server.cpp implements Dev with HIP; a CPU test double implements it with
// scripted searches, so that admission, retries, completion order and the
// latency accounting can be checked (also under ThreadSanitizer) without a
// GPU.  Nothing here includes HIP.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "rr.h"

namespace rr {

struct ServerRequest {
    uint64_t tag = 0;
    double radius = 0;
    double t_arrival = 0;
    std::vector<uint8_t> q;
    bool solo = false; // run in a tick of its own (a retry after a shared capacity ran out)
    int32_t ticks = 0; // ticks already spent (a retry keeps counting)
};

struct ServerFinished {
    std::vector<int32_t> ids;
    std::vector<uint8_t> dists; // int32 (integer data) or float32 (float data)
};

struct SlotOutcome {
    bool done = false;
    rr_query_stats stats{};
};

template <class Dev> class ServerCore {
  public:
    using Clock = std::chrono::steady_clock;

    ServerCore(Dev &dev, int32_t S, int32_t max_pending, int64_t qbytes)
        : dev_(dev), S_(S), max_pending_(max_pending), qbytes_(qbytes), t0_(Clock::now()) {
        slots_.assign((size_t)S, Slot());
        free_slots_.reserve((size_t)S);
        for (int64_t i = (int64_t)S - 1; i >= 0; --i) free_slots_.push_back((int32_t)i);
        info_.slots = S;
    }
    ServerCore(const ServerCore &) = delete;
    ServerCore &operator=(const ServerCore &) = delete;
    ~ServerCore() { stop(); }

    // starts the worker; `thread_init` runs first on the worker thread
    // (device selection) and may fail with a message
    bool start(std::function<bool(std::string &)> thread_init) {
        try {
            worker_ = std::thread([this, thread_init] { worker_main(thread_init); });
        } catch (...) {
            return false;
        }
        return true;
    }

    // lets the queued and resident requests finish, then ends the worker
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (worker_.joinable()) worker_.join();
    }

    double now() const { return std::chrono::duration<double>(Clock::now() - t0_).count(); }

    void set_device_bytes(int64_t b) {
        std::lock_guard<std::mutex> lk(mu_);
        info_.device_bytes = b;
    }

    rr_status submit(const void *query, double radius, uint64_t tag, double t_arrival, std::string &msg) {
        ServerRequest r;
        r.tag = tag;
        r.radius = radius;
        r.q.assign((const uint8_t *)query, (const uint8_t *)query + qbytes_);
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (failed_) return (msg = error_, RR_ESTATE);
            if (stop_) return (msg = "server is stopping", RR_ESTATE);
            if ((int64_t)pending_.size() >= max_pending_)
                return (msg = "request queue is full (" + std::to_string(max_pending_) + ")", RR_EBUSY);
            r.t_arrival = t_arrival >= 0 ? t_arrival : now();
            pending_.push_back(std::move(r));
            info_.submitted += 1;
            info_.pending = (int64_t)pending_.size();
        }
        cv_work_.notify_one();
        return RR_OK;
    }

    rr_status poll(rr_completion *out, int32_t max, int32_t *n, std::string &msg) {
        std::lock_guard<std::mutex> lk(mu_);
        int32_t k = 0;
        while (k < max && !completions_.empty()) {
            out[k++] = completions_.front();
            completions_.pop_front();
        }
        *n = k;
        if (failed_) return (msg = error_, RR_ESTATE);
        return RR_OK;
    }

    rr_status result(uint64_t tag, int32_t *ids, void *dists, int64_t capacity, int64_t *count,
                     std::string &msg) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = results_.find(tag);
        if (it == results_.end()) return (msg = "no finished request with this tag", RR_EINVAL);
        const int64_t c = (int64_t)it->second.ids.size();
        *count = c;
        if (capacity < c)
            return (msg = "capacity " + std::to_string(capacity) + " < " + std::to_string(c) + " results",
                    RR_ENOMEM);
        if (c > 0 && (!ids || !dists)) return (msg = "output buffers are NULL", RR_EINVAL);
        if (c > 0) {
            std::memcpy(ids, it->second.ids.data(), (size_t)c * 4);
            std::memcpy(dists, it->second.dists.data(), (size_t)c * 4);
        }
        results_.erase(it);
        return RR_OK;
    }

    rr_status drain(double timeout_s, std::string &msg) {
        std::unique_lock<std::mutex> lk(mu_);
        auto idle = [&] { return failed_ || (pending_.empty() && info_.completed == info_.submitted); };
        if (timeout_s < 0) {
            cv_done_.wait(lk, idle);
        } else {
            // a system_clock deadline: a steady_clock wait goes through
            // pthread_cond_clockwait, which ThreadSanitizer (gcc 11) does not
            // intercept, so it would report the mutex as never released
            const auto until = std::chrono::system_clock::now() +
                               std::chrono::duration_cast<std::chrono::system_clock::duration>(
                                   std::chrono::duration<double>(timeout_s));
            if (!cv_done_.wait_until(lk, until, idle)) return (msg = "drain timed out", RR_EBUSY);
        }
        if (failed_) return (msg = error_, RR_ESTATE);
        return RR_OK;
    }

    rr_server_info info() const {
        std::lock_guard<std::mutex> lk(mu_);
        return info_;
    }

  private:
    struct Slot {
        bool busy = false;
        bool solo = false;
        uint64_t tag = 0;
        double radius = 0;
        double t_arrival = 0, t_admit = 0;
        int32_t ticks = 0;
        std::vector<uint8_t> q; // the request's vector, kept for a retry
    };

    void fail(const std::string &why) {
        std::lock_guard<std::mutex> lk(mu_);
        failed_ = true;
        error_ = why;
        cv_done_.notify_all();
    }

    void worker_main(std::function<bool(std::string &)> thread_init) {
        {
            std::string why;
            if (thread_init && !thread_init(why)) {
                fail(why);
                return;
            }
        }
        std::vector<int32_t> active;
        active.reserve((size_t)S_);
        for (;;) {
            int32_t admitted = 0;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_work_.wait(lk, [&] {
                    return stop_ || !active.empty() || (!pending_.empty() && !free_slots_.empty());
                });
                if (stop_ && pending_.empty() && active.empty()) break;
                const double t = now();
                while (!pending_.empty() && !free_slots_.empty()) {
                    ServerRequest &r = pending_.front();
                    // a retry runs alone: it waits until nothing else is
                    // resident, and nothing else joins its tick
                    if (r.solo && (!active.empty() || admitted > 0)) break;
                    if (!active.empty() && slots_[(size_t)active[0]].solo) break;
                    const int32_t slot = free_slots_.back();
                    free_slots_.pop_back();
                    dev_.stage(admitted, slot, r);
                    Slot &sl = slots_[(size_t)slot];
                    sl.busy = true;
                    sl.solo = r.solo;
                    sl.tag = r.tag;
                    sl.radius = r.radius;
                    sl.t_arrival = r.t_arrival;
                    if (!r.solo) sl.t_admit = t;
                    sl.ticks = r.ticks;
                    sl.q.swap(r.q);
                    active.push_back(slot);
                    ++admitted;
                    pending_.pop_front();
                    if (sl.solo) break;
                }
                info_.admitted += admitted;
                info_.pending = (int64_t)pending_.size();
                info_.resident = (int64_t)active.size();
                info_.max_resident = std::max<int64_t>(info_.max_resident, (int64_t)active.size());
            }
            const Clock::time_point tb = Clock::now();
            std::string why;
            if (!dev_.tick(admitted, active.data(), (int32_t)active.size(), why)) {
                fail("server tick failed: " + why);
                return;
            }
            // collect the slots whose search finished in this tick.  The
            // greedy items, the (task, id) set and the result capacity are
            // shared by the tick's queries; when one of them ran out, a query
            // flagged truncated may only have lost results to its neighbours,
            // so it runs again in a tick of its own.  A query truncated alone
            // is returned truncated.
            const bool shared_overflow = dev_.shared_overflow();
            std::vector<rr_completion> done;
            std::vector<std::pair<uint64_t, ServerFinished>> out;
            std::vector<int32_t> freed;
            std::vector<ServerRequest> retry;
            size_t keep = 0;
            for (size_t i = 0; i < active.size(); ++i) {
                const int32_t slot = active[i];
                Slot &sl = slots_[(size_t)slot];
                ++sl.ticks;
                const SlotOutcome oc = dev_.outcome(slot);
                if (!oc.done) {
                    active[keep++] = slot;
                    continue;
                }
                if (oc.stats.truncated && shared_overflow && !sl.solo) {
                    ServerRequest r;
                    r.tag = sl.tag;
                    r.radius = sl.radius;
                    r.t_arrival = sl.t_arrival;
                    r.q.swap(sl.q);
                    r.solo = true;
                    r.ticks = sl.ticks;
                    retry.push_back(std::move(r));
                    freed.push_back(slot);
                    sl.busy = false;
                    continue;
                }
                ServerFinished f;
                if (!dev_.result(slot, f, why)) {
                    fail(why);
                    return;
                }
                rr_completion c{};
                c.tag = sl.tag;
                c.count = (int32_t)f.ids.size();
                c.stats = oc.stats;
                c.truncated = oc.stats.truncated;
                c.ticks = sl.ticks;
                c.t_arrival = sl.t_arrival;
                c.t_admit = sl.t_admit;
                done.push_back(c);
                out.emplace_back(sl.tag, std::move(f));
                freed.push_back(slot);
                sl.busy = false;
                sl.solo = false;
                sl.q.clear();
            }
            active.resize(keep);
            const double t = now();
            {
                std::lock_guard<std::mutex> lk(mu_);
                for (size_t i = 0; i < done.size(); ++i) {
                    done[i].t_done = t;
                    results_[done[i].tag] = std::move(out[i].second);
                    completions_.push_back(done[i]);
                }
                for (int32_t f : freed) free_slots_.push_back(f);
                // retries go first, in their original order
                for (size_t i = retry.size(); i-- > 0;) pending_.push_front(std::move(retry[i]));
                info_.retried += (int64_t)retry.size();
                info_.completed += (int64_t)done.size();
                info_.ticks += 1;
                info_.resident = (int64_t)active.size();
                const double tick_s = std::chrono::duration<double>(Clock::now() - tb).count();
                info_.busy_s += tick_s;
                info_.max_tick_s = std::max(info_.max_tick_s, tick_s);
                cv_done_.notify_all();
            }
        }
        std::lock_guard<std::mutex> lk(mu_);
        cv_done_.notify_all();
    }

    Dev &dev_;
    const int32_t S_;
    const int64_t max_pending_;
    const int64_t qbytes_;
    const Clock::time_point t0_;
    std::thread worker_;
    mutable std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    bool stop_ = false;
    bool failed_ = false;
    std::string error_;
    std::deque<ServerRequest> pending_;
    std::vector<Slot> slots_;
    std::vector<int32_t> free_slots_;
    std::deque<rr_completion> completions_;
    std::unordered_map<uint64_t, ServerFinished> results_;
    rr_server_info info_{};
};

} // namespace rr
