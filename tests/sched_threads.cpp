// Many threads against the scheduler service (the serving loop's locking and
// worker thread) with a fake executor whose batches take wall-clock time:
// 8 producers submit, 2 clients take completions and release them, a reader
// polls statistics.  Built with g++ (plain, ThreadSanitizer, ASan + UBSan)
// by tests/test_scheduler.py.  Every request must complete exactly once, the
// budget must come back whole, and the counters must agree.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../paper_2005_08165_amd/csrc/sne_sched.h"

using namespace sne::sched;
using Clock = std::chrono::steady_clock;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);             \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

// Called only from the service's worker thread (under its lock); a batch
// finishes 20 us + 1 ns per pixel after its launch.
struct WallExec : Executor {
    Clock::time_point t0 = Clock::now();
    std::vector<double> end_of;
    int launches = 0;
    explicit WallExec(int slots) : end_of(slots, 0.0) {}
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    int launch(Batch &b) override {
        ++launches;
        end_of[b.slot] = now() + 20e-6 + 1e-9 * (double)b.pixels;
        return 0;
    }
    bool done(const Batch &b) override { return now() >= end_of[b.slot]; }
};

int main() {
    const int kProducers = 8, kPerProducer = 400, kClients = 2;
    Config cfg;
    cfg.max_inflight = 3;
    cfg.max_batch_frames = 16;
    cfg.budget_bytes = 64ull << 20;
    cfg.align = 256;
    cfg.queue_capacity = 1 << 20;
    WallExec ex(cfg.max_inflight);
    Service svc(cfg, &ex, [&ex] { return ex.now(); });

    std::atomic<int> submitted{0}, completed{0}, producers_done{0};
    std::mutex seen_mu;
    std::set<uint64_t> seen;
    std::vector<std::thread> th;
    for (int p = 0; p < kProducers; ++p)
        th.emplace_back([&, p] {
            std::mt19937 rng(1000 + p);
            for (int i = 0; i < kPerProducer; ++i) {
                Request r;
                r.stream = p;
                r.H = 8 + (int)(rng() % 120);
                r.W = 8 + (int)(rng() % 160);
                r.out_bytes = (uint64_t)r.H * r.W * 7;
                r.t_arrival = -1.0;
                uint64_t t = 0;
                int rc;
                while ((rc = svc.submit(r, &t)) == -6) std::this_thread::yield();
                CHECK(rc == 0 && t != 0);
                submitted.fetch_add(1);
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(30));
            }
            producers_done.fetch_add(1);
        });
    for (int c = 0; c < kClients; ++c)
        th.emplace_back([&] {
            while (completed.load() < kProducers * kPerProducer) {
                std::vector<Request> done = svc.take_completed(64);
                for (const Request &q : done) {
                    CHECK(q.status == 0 && q.finished);
                    CHECK(q.t_arrival <= q.t_launch && q.t_launch <= q.t_done);
                    {
                        std::lock_guard<std::mutex> lk(seen_mu);
                        CHECK(seen.insert(q.ticket).second);  // each ticket once
                    }
                    CHECK(svc.release(q.ticket) == 0);
                    CHECK(svc.release(q.ticket) != 0);       // not twice
                    completed.fetch_add(1);
                }
                if (done.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        });
    th.emplace_back([&] {  // statistics while everything moves
        while (producers_done.load() < kProducers) {
            const uint64_t sub = svc.inspect([](const Scheduler &s) { return s.stats().submitted; });
            CHECK(sub <= (uint64_t)kProducers * kPerProducer);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
    });
    for (auto &t : th) t.join();
    CHECK(svc.drain(10.0));
    CHECK(submitted.load() == kProducers * kPerProducer);
    CHECK(completed.load() == kProducers * kPerProducer && (int)seen.size() == completed.load());
    const bool ok = svc.inspect([&](const Scheduler &s) {
        const Stats &st = s.stats();
        return st.submitted == (uint64_t)submitted.load() &&
               st.completed == (uint64_t)completed.load() && st.failed == 0 &&
               st.frames_in_batches == st.completed && s.arena_free() == cfg.budget_bytes &&
               s.idle();
    });
    CHECK(ok);
    svc.stop();
    std::printf("ok service: %d requests from %d threads, %d batches\n", completed.load(),
                kProducers, ex.launches);
    std::printf("ALL OK\n");
    return 0;
}
