// CPU test double of the serving loop: rr::ServerCore (the host side of
// rr_server_*) driven by a scripted device instead of the GPU, under the
// sanitizers.  Test infrastructure only.
//
// Each request's first bytes script its search: q[0] % 4 + 1 ticks until its
// beam search finishes, q[1] results, q[2] != 0 "heavy".  Heavy requests that
// finish in the same tick exceed a capacity they share: the fake device flags
// them truncated and reports the overflow, so the core must run each of them
// again alone (a tick holding a retried request holds nothing else; the fake
// device fails the tick otherwise) and return it complete.  Four threads
// submit while one polls; every request must come back exactly once, with
// its full result, with t_arrival <= t_admit <= t_done, after at least its
// scripted number of ticks, and the counters must agree.
//
// usage: server_double [requests_per_thread]   (exit 0 and "OK" on success)
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rr_server_core.h"

namespace {

constexpr int S = 8;
constexpr int QBYTES = 16;

struct FakeDev {
    struct Slot {
        uint64_t tag = 0;
        int need = 0, progress = 0, count = 0;
        bool heavy = false, solo = false, finished = false, truncated = false;
    };
    std::vector<Slot> slots = std::vector<Slot>(S);
    bool overflow = false;
    int64_t solo_ticks = 0, ticks = 0;

    bool stage(int32_t, int32_t slot, const rr::ServerRequest &r) {
        Slot &s = slots[(size_t)slot];
        s = Slot();
        s.tag = r.tag;
        s.need = r.q[0] % 4 + 1;
        s.count = r.q[1];
        s.heavy = r.q[2] != 0;
        s.solo = r.solo;
        return true;
    }
    bool tick(int32_t, const int32_t *active, int32_t nwork, std::string &err) {
        ++ticks;
        int heavy_done = 0;
        for (int32_t i = 0; i < nwork; ++i) {
            Slot &s = slots[(size_t)active[i]];
            if (s.solo) {
                ++solo_ticks;
                if (nwork != 1) {
                    err = "a retried request shares its tick";
                    return false;
                }
            }
            s.finished = ++s.progress >= s.need;
            s.truncated = false;
            if (s.finished && s.heavy) ++heavy_done;
        }
        overflow = heavy_done >= 2;
        if (overflow)
            for (int32_t i = 0; i < nwork; ++i) {
                Slot &s = slots[(size_t)active[i]];
                if (s.finished && s.heavy) s.truncated = true;
            }
        std::this_thread::sleep_for(std::chrono::microseconds(50 + 10 * nwork));
        return true;
    }
    rr::SlotOutcome outcome(int32_t slot) const {
        const Slot &s = slots[(size_t)slot];
        rr::SlotOutcome oc;
        oc.done = s.finished;
        oc.stats.truncated = s.truncated ? 1 : 0;
        oc.stats.visits = s.progress;
        return oc;
    }
    bool shared_overflow() const { return overflow; }
    bool result(int32_t slot, rr::ServerFinished &f, std::string &) const {
        const Slot &s = slots[(size_t)slot];
        const int n = s.truncated ? s.count / 2 : s.count;
        f.ids.resize((size_t)n);
        f.dists.resize((size_t)n * 4);
        for (int j = 0; j < n; ++j) {
            f.ids[(size_t)j] = (int32_t)((s.tag * 7 + (uint64_t)j) & 0x7fffffff);
            const int32_t d = j;
            std::memcpy(f.dists.data() + 4 * (size_t)j, &d, 4);
        }
        return true;
    }
};

struct Script {
    uint8_t need, count, heavy;
};

#define CHECK(c)                                                                            \
    do {                                                                                    \
        if (!(c)) {                                                                         \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);          \
            std::exit(1);                                                                   \
        }                                                                                   \
    } while (0)

} // namespace

int main(int argc, char **argv) {
    const int per_thread = argc > 1 ? std::atoi(argv[1]) : 400;
    constexpr int THREADS = 4;
    const int total = per_thread * THREADS;
    FakeDev dev;
    rr::ServerCore<FakeDev> core(dev, S, 1 << 20, QBYTES);
    CHECK(core.start([](std::string &) { return true; }));

    std::mutex script_mu;
    std::unordered_map<uint64_t, Script> script;
    std::vector<std::thread> submitters;
    for (int t = 0; t < THREADS; ++t) {
        submitters.emplace_back([&, t] {
            std::mt19937 rng(1234 + t);
            for (int i = 0; i < per_thread; ++i) {
                uint8_t q[QBYTES] = {0};
                q[0] = (uint8_t)(rng() % 4);
                q[1] = (uint8_t)(rng() % 40);
                q[2] = (uint8_t)(rng() % 5 == 0);
                const uint64_t tag = (uint64_t)t * 1000000 + (uint64_t)i;
                {
                    std::lock_guard<std::mutex> lk(script_mu);
                    script[tag] = Script{(uint8_t)(q[0] + 1), q[1], q[2]};
                }
                std::string msg;
                CHECK(core.submit(q, 1.0, tag, -1.0, msg) == RR_OK);
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
            }
        });
    }

    std::set<uint64_t> seen;
    int64_t got = 0;
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(120);
    std::vector<rr_completion> buf(64);
    std::vector<int32_t> ids(256);
    std::vector<int32_t> dists(256);
    while (got < total) {
        CHECK(std::chrono::steady_clock::now() < deadline);
        int32_t n = 0;
        std::string msg;
        CHECK(core.poll(buf.data(), (int32_t)buf.size(), &n, msg) == RR_OK);
        for (int32_t k = 0; k < n; ++k) {
            const rr_completion &c = buf[(size_t)k];
            CHECK(seen.insert(c.tag).second); // exactly once
            Script sc;
            {
                std::lock_guard<std::mutex> lk(script_mu);
                auto it = script.find(c.tag);
                CHECK(it != script.end());
                sc = it->second;
            }
            CHECK(!c.truncated);
            CHECK(c.count == sc.count);
            CHECK(c.ticks >= sc.need);
            CHECK(c.t_arrival <= c.t_admit && c.t_admit <= c.t_done);
            int64_t cnt = 0;
            CHECK(core.result(c.tag, ids.data(), dists.data(), (int64_t)ids.size(), &cnt, msg) == RR_OK);
            CHECK(cnt == sc.count);
            for (int64_t j = 0; j < cnt; ++j) {
                CHECK(ids[(size_t)j] == (int32_t)((c.tag * 7 + (uint64_t)j) & 0x7fffffff));
                CHECK(dists[(size_t)j] == (int32_t)j);
            }
            CHECK(core.result(c.tag, ids.data(), dists.data(), (int64_t)ids.size(), &cnt, msg) == RR_EINVAL);
            ++got;
        }
        if (n == 0) std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    for (auto &th : submitters) th.join();
    std::string msg;
    CHECK(core.drain(10.0, msg) == RR_OK);
    const rr_server_info info = core.info();
    CHECK(info.submitted == total && info.completed == total && info.admitted >= total);
    CHECK(info.admitted == total + info.retried);
    CHECK(info.pending == 0 && info.resident == 0 && info.max_resident <= S && info.max_resident >= 2);
    CHECK(info.retried > 0);
    CHECK(info.ticks == dev.ticks);
    CHECK(dev.solo_ticks > 0);
    // a full queue is refused, not dropped
    {
        FakeDev dev2;
        rr::ServerCore<FakeDev> small(dev2, S, 2, QBYTES);
        uint8_t q[QBYTES] = {0};
        CHECK(small.submit(q, 1.0, 1, -1.0, msg) == RR_OK);
        CHECK(small.submit(q, 1.0, 2, -1.0, msg) == RR_OK);
        CHECK(small.submit(q, 1.0, 3, -1.0, msg) == RR_EBUSY);
        CHECK(small.start([](std::string &) { return true; }));
        CHECK(small.drain(10.0, msg) == RR_OK);
        CHECK(small.info().completed == 2);
    }
    // a failing thread start is reported to every caller
    {
        FakeDev dev3;
        rr::ServerCore<FakeDev> bad(dev3, S, 16, QBYTES);
        CHECK(bad.start([](std::string &why) {
            why = "no device";
            return false;
        }));
        // the failure is reported once the worker has run: submissions are
        // refused from then on, and drain and poll report it
        uint8_t q[QBYTES] = {0};
        rr_status st = RR_OK;
        for (int i = 0; i < 100000 && st == RR_OK; ++i) {
            st = bad.submit(q, 1.0, (uint64_t)i, -1.0, msg);
            if (st == RR_OK) std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(st == RR_ESTATE && msg == "no device");
        CHECK(bad.drain(10.0, msg) == RR_ESTATE && msg == "no device");
        int32_t n = 0;
        CHECK(bad.poll(buf.data(), 1, &n, msg) == RR_ESTATE && n == 0);
    }
    std::printf("OK requests %d ticks %lld retried %lld solo ticks %lld max resident %lld\n", total,
                (long long)info.ticks, (long long)info.retried, (long long)dev.solo_ticks,
                (long long)info.max_resident);
    return 0;
}
