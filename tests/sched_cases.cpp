// Unit cases for the continuous-batching scheduler core, driven by a fake
// executor on a simulated clock.  Built with g++ and run by
// tests/test_scheduler.py; prints one line per case and exits non-zero on
// the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>

#include "../paper_2005_08165_amd/csrc/sne_sched.h"

using namespace sne::sched;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);             \
            std::exit(1);                                                        \
        }                                                                        \
    } while (0)

// A batch takes `overhead + pixels / rate` seconds of simulated time; launch
// may be told to fail.
struct FakeExec : Executor {
    double *clock;
    double overhead, rate;
    int fail_next = 0;
    int launches = 0;
    int max_concurrent = 0;
    std::vector<double> end_of;  // per slot
    std::vector<std::vector<uint64_t>> history;
    FakeExec(double *c, int slots, double oh, double r)
        : clock(c), overhead(oh), rate(r), end_of(slots, -1.0) {}
    int launch(Batch &b) override {
        ++launches;
        if (fail_next > 0) {
            --fail_next;
            return -4;
        }
        end_of[b.slot] = *clock + overhead + (double)b.pixels / rate;
        std::vector<uint64_t> t;
        for (auto *q : b.reqs) t.push_back(q->ticket);
        history.push_back(t);
        int n = 0;
        for (double e : end_of) n += e > *clock ? 1 : 0;
        if (n > max_concurrent) max_concurrent = n;
        return 0;
    }
    bool done(const Batch &b) override { return *clock >= end_of[b.slot]; }
};

static Request req(int H, int W, double t, int stream = 0) {
    Request r;
    r.H = H;
    r.W = W;
    r.stream = stream;
    r.out_bytes = (uint64_t)H * W * 13;  // fp32 normals + mask
    r.t_arrival = t;
    return r;
}

static void case_arena() {
    Arena a(1024, 64);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);   // rounds to 128
    CHECK(a.alloc(64, &o2) && o2 == 128);
    CHECK(a.alloc(800, &o3) && o3 == 192);
    CHECK(!a.alloc(64, &o4));              // 32 bytes left
    a.release(o2, 64);
    CHECK(a.alloc(60, &o4) && o4 == 128);  // reuses the hole
    a.release(o1, 100);
    a.release(o4, 60);
    a.release(o3, 800);
    CHECK(a.free_bytes() == 1024);
    CHECK(a.alloc(1024, &o1) && o1 == 0);  // fully coalesced
    std::printf("ok arena\n");
}

static void case_continuous_batching() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 2;
    cfg.max_batch_frames = 8;
    cfg.budget_bytes = 1ull << 30;
    FakeExec ex(&clock, 2, 1e-4, 1e9);
    Scheduler s(cfg, &ex);
    // 20 requests arriving every 10 us while batches take ~100 us
    std::vector<uint64_t> tickets;
    int next = 0;
    for (int tick = 0; tick < 2000 && (next < 20 || !s.idle()); ++tick) {
        clock = tick * 1e-5;
        while (next < 20 && next * 1e-5 <= clock) {
            uint64_t t;
            CHECK(s.submit(req(100, 100, clock), &t) == 0);
            tickets.push_back(t);
            ++next;
        }
        s.step(clock);
        for (auto &r : s.take_completed(100)) CHECK(s.release(r.ticket) == 0);
    }
    CHECK(s.idle());
    CHECK(s.stats().completed == 20);
    CHECK(ex.max_concurrent == 2);            // batches overlapped
    CHECK(s.stats().batches < 20);            // requests were grouped
    // arrivals during a running batch joined a later batch, in order
    std::vector<uint64_t> order;
    for (auto &b : ex.history)
        for (auto t : b) order.push_back(t);
    for (size_t i = 1; i < order.size(); ++i) CHECK(order[i] > order[i - 1]);
    CHECK(s.arena_free() == cfg.budget_bytes);
    std::printf("ok continuous_batching batches=%llu\n", (unsigned long long)s.stats().batches);
}

static void case_budget_admission_fifo() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 4;
    cfg.budget_bytes = 3 * 100 * 100 * 13 + 100;  // room for three 100x100 frames
    cfg.align = 1;
    FakeExec ex(&clock, 4, 1e-3, 1e12);
    Scheduler s(cfg, &ex);
    uint64_t t[6];
    for (int i = 0; i < 6; ++i) CHECK(s.submit(req(100, 100, 0.0), &t[i]) == 0);
    s.step(0.0);
    CHECK(s.waiting() == 3);                  // only three fit the budget
    clock = 0.002;
    s.step(clock);
    auto done = s.take_completed(10);
    CHECK(done.size() == 3);
    s.step(clock);
    CHECK(s.waiting() == 3);                  // outputs still held by the client
    for (auto &r : done) CHECK(s.release(r.ticket) == 0);
    s.step(clock);
    CHECK(s.waiting() == 0);                  // released budget admits the rest
    // a frame larger than the whole budget is rejected outright
    uint64_t big;
    CHECK(s.submit(req(1000, 1000, clock), &big) == -3);
    CHECK(s.stats().rejected_budget == 1);
    std::printf("ok budget_admission_fifo\n");
}

static void case_no_starvation() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 1;
    cfg.budget_bytes = 2 * 400 * 400 * 13;
    cfg.align = 1;
    FakeExec ex(&clock, 1, 1e-4, 1e9);
    Scheduler s(cfg, &ex);
    uint64_t big = 0;
    // a stream of small frames with one large frame in the middle: the large
    // frame must be served although small ones keep arriving
    int n = 0;
    bool big_done = false;
    for (int tick = 0; tick < 20000 && !big_done; ++tick) {
        clock = tick * 1e-5;
        if (tick % 3 == 0) {
            uint64_t t;
            CHECK(s.submit(req(200, 200, clock), &t) == 0);
            ++n;
        }
        if (tick == 30) CHECK(s.submit(req(400, 400, clock), &big) == 0);
        s.step(clock);
        for (auto &r : s.take_completed(100)) {
            if (r.ticket == big) big_done = true;
            CHECK(s.release(r.ticket) == 0);
        }
    }
    CHECK(big_done);
    std::printf("ok no_starvation\n");
}

static void case_backpressure() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 1;
    cfg.queue_capacity = 5;
    FakeExec ex(&clock, 1, 1.0, 1e9);
    Scheduler s(cfg, &ex);
    uint64_t t;
    for (int i = 0; i < 5; ++i) CHECK(s.submit(req(10, 10, 0), &t) == 0);
    CHECK(s.submit(req(10, 10, 0), &t) == -6);
    CHECK(s.stats().rejected_full == 1);
    s.step(0);  // launches: the queue drains into the slot
    CHECK(s.submit(req(10, 10, 0), &t) == 0);
    std::printf("ok backpressure\n");
}

static void case_executor_failure() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 1;
    cfg.max_batch_frames = 2;
    FakeExec ex(&clock, 1, 1e-4, 1e9);
    Scheduler s(cfg, &ex);
    uint64_t t;
    for (int i = 0; i < 6; ++i) CHECK(s.submit(req(10, 10, 0), &t) == 0);
    ex.fail_next = 1;
    int failed = 0, ok = 0;
    for (int tick = 0; tick < 1000 && !s.idle(); ++tick) {
        clock = tick * 1e-4;
        s.step(clock);
        for (auto &r : s.take_completed(100)) {
            (r.status == 0 ? ok : failed)++;
            CHECK(s.release(r.ticket) == 0);
        }
    }
    CHECK(failed == 2 && ok == 4);            // one batch failed, the loop went on
    CHECK(s.stats().failed == 2 && s.stats().completed == 4);
    CHECK(s.arena_free() == cfg.budget_bytes);
    std::printf("ok executor_failure\n");
}

static void case_batch_limits() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 1;
    cfg.max_batch_frames = 4;
    cfg.max_batch_pixels = 250;
    FakeExec ex(&clock, 1, 1e-4, 1e12);
    Scheduler s(cfg, &ex);
    uint64_t t;
    for (int i = 0; i < 6; ++i) CHECK(s.submit(req(10, 10, 0), &t) == 0);  // 100 px each
    s.step(0);
    CHECK(ex.history.size() == 1 && ex.history[0].size() == 2);  // pixel cap
    CHECK(s.submit(req(30, 30, 0), &t) == 0);  // 900 px: over the cap, still served alone
    for (int tick = 1; tick < 100 && !s.idle(); ++tick) {
        clock = tick * 1e-3;
        s.step(clock);
        for (auto &r : s.take_completed(100)) s.release(r.ticket);
    }
    CHECK(s.idle());
    bool alone = false;
    for (auto &b : ex.history) alone = alone || (b.size() == 1);
    CHECK(alone);
    std::printf("ok batch_limits\n");
}

static void case_release_rules() {
    double clock = 0;
    Config cfg;
    cfg.max_inflight = 1;
    FakeExec ex(&clock, 1, 1.0, 1e9);
    Scheduler s(cfg, &ex);
    uint64_t t;
    CHECK(s.submit(req(10, 10, 0), &t) == 0);
    s.step(0);
    CHECK(s.release(t) == -5);                // running: cannot release
    CHECK(s.release(12345) == -1);            // unknown ticket
    clock = 2.0;
    s.step(clock);
    CHECK(s.release(t) == 0);
    CHECK(s.release(t) == -1);                // already released
    std::printf("ok release_rules\n");
}

static void case_quantile() {
    std::vector<double> v;
    for (int i = 1; i <= 100; ++i) v.push_back(i);
    CHECK(quantile(v, 0.5) == 51);
    CHECK(quantile(v, 0.99) == 100);
    CHECK(quantile(v, 0.0) == 1);
    CHECK(quantile({}, 0.5) == 0);
    std::printf("ok quantile\n");
}

// The fixed-memory latency histogram agrees with exact nearest-rank
// quantiles within its 1 % bins, keeps the exact maximum, and a long run adds
// no memory (the latencies are not stored).
static void case_latency_histogram() {
    std::mt19937_64 g(7);
    std::lognormal_distribution<double> d(std::log(400e-6), 0.8);
    LatencyHistogram h;
    std::vector<double> v;
    for (int i = 0; i < 200000; ++i) {
        const double x = d(g);
        h.add(x);
        v.push_back(x);
    }
    CHECK(h.count() == v.size());
    for (double q : {0.0, 0.1, 0.5, 0.9, 0.99, 0.999, 1.0}) {
        const double exact = quantile(v, q), got = h.quantile(q);
        CHECK(got >= exact * (1 - 1e-12) && got <= exact * 1.0101);
    }
    CHECK(h.max() == quantile(v, 1.0));
    LatencyHistogram e;
    CHECK(e.quantile(0.5) == 0 && e.max() == 0);
    e.add(0.0);
    e.add(-1.0);                                // clock skew: counted as 0
    e.add(1e9);                                 // beyond the last bin
    CHECK(e.count() == 3 && e.max() == 1e9 && e.quantile(0.0) == 0.0);
    std::printf("ok latency_histogram\n");
}

int main() {
    case_latency_histogram();
    case_arena();
    case_continuous_batching();
    case_budget_admission_fifo();
    case_no_starvation();
    case_backpressure();
    case_executor_failure();
    case_batch_limits();
    case_release_rules();
    case_quantile();
    std::printf("ALL OK\n");
    return 0;
}
