// sne_sched.h - continuous-batching scheduler core of the serving loop.
//
// Pure C++ (no HIP): the server drives it with a HIP executor, the capacity
// simulator and the CPU tests drive it with a fake executor on a simulated
// clock.  Not part of the public ABI.
//
// Model.  Requests (one frame each) arrive over time.  A request is ADMITTED
// when its output bytes fit in the HBM budget that completed-but-unreleased
// and in-flight outputs leave free; admission is FIFO over arrival order (a
// large frame at the head waits for memory rather than being overtaken, so
// nothing starves).  Whenever an in-flight slot is free and admitted requests
// are waiting, a batch is formed from them (up to max_batch_frames frames and
// max_batch_pixels pixels, in order) and handed to the executor on that slot.
// Batches on different slots overlap on the device; requests that arrive
// while batches run join the next batch.  A completed batch frees its slot;
// a request's budget is returned when the client releases its output.
#pragma once

#include <stdint.h>

#include <atomic>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace sne {
namespace sched {

struct Request {
    uint64_t ticket = 0;
    int32_t stream = 0;
    int32_t H = 0, W = 0;
    uint64_t out_bytes = 0;   // normals + mask
    double t_arrival = 0.0;   // seconds, scheduler clock
    double t_admit = 0.0, t_launch = 0.0, t_done = 0.0;
    uint64_t out_offset = 0;  // offset of the request's outputs in the arena
    bool has_output = false;  // out_offset holds an arena allocation
    bool finished = false;    // completed or failed
    int status = 0;
    const void *in = nullptr;  // the frame (read by the executor only)
    int64_t in_pitch = 0;      // its row pitch in elements
    const void *ready = nullptr;  // event the frame's producer recorded, or null
};

struct Config {
    int max_inflight = 3;            // concurrent batches (slots)
    int max_batch_frames = 256;
    uint64_t max_batch_pixels = 64ull << 20;
    uint64_t budget_bytes = 4ull << 30;  // output arena size
    uint64_t align = 256;            // output allocation granularity
    size_t queue_capacity = 65536;   // waiting + admitted requests
};

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
public:
    explicit Arena(uint64_t size = 0, uint64_t align = 256);
    bool alloc(uint64_t bytes, uint64_t *offset);
    void release(uint64_t offset, uint64_t bytes);
    uint64_t free_bytes() const { return free_; }
    uint64_t size() const { return size_; }
    uint64_t round(uint64_t b) const { return (b + align_ - 1) / align_ * align_; }

private:
    std::map<uint64_t, uint64_t> holes_;  // offset -> length
    uint64_t size_, align_, free_;
};

// A batch handed to the executor.
struct Batch {
    int slot = -1;
    std::vector<Request *> reqs;
    uint64_t pixels = 0;
};

// The executor launches a batch on a slot and later reports whether it has
// finished.  launch() returns 0 on success; a failure fails every request of
// the batch and frees the slot.
struct Executor {
    virtual ~Executor() {}
    virtual int launch(Batch &b) = 0;
    virtual bool done(const Batch &b) = 0;  // non-blocking
    virtual int result(const Batch &b) { (void)b; return 0; }
};

// Latency distribution in fixed memory: logarithmic bins 1 % wide from
// 0.1 us to 10^4 s, so a server can run indefinitely.  Quantiles are exact to
// the bin (within 1 %), clamped to the exact minimum and maximum.
class LatencyHistogram {
public:
    LatencyHistogram();
    void add(double seconds);
    uint64_t count() const { return n_; }
    double max() const { return n_ ? max_ : 0.0; }
    // nearest-rank quantile, q in [0, 1]; 0 if empty
    double quantile(double q) const;

private:
    std::vector<uint64_t> bins_;
    uint64_t n_ = 0;
    double min_ = 0.0, max_ = 0.0;
};

struct Stats {
    uint64_t submitted = 0, rejected_full = 0, rejected_budget = 0, completed = 0, failed = 0;
    uint64_t batches = 0, frames_in_batches = 0, pixels_done = 0;
    double first_arrival = 0.0, last_done = 0.0;
    LatencyHistogram latency;  // t_done - t_arrival of completed requests
};

class Scheduler {
public:
    Scheduler(const Config &cfg, Executor *ex);
    ~Scheduler();

    // Enqueue a request (t_arrival is taken from the request).  Returns
    // 0, -3 (a single frame larger than the whole budget) or -6 (queue full).
    int submit(const Request &r, uint64_t *ticket);
    // One scheduling pass at time `now`: retire finished batches, admit,
    // launch.  Returns the number of batches launched.
    int step(double now);
    // Completed requests not yet taken by the client (moved out).
    std::vector<Request> take_completed(size_t max);
    // Return a completed request's outputs to the budget.
    int release(uint64_t ticket);

    size_t waiting() const { return waiting_.size(); }
    size_t admitted() const { return admitted_.size(); }
    int inflight() const;
    bool idle() const { return waiting_.empty() && admitted_.empty() && inflight() == 0; }
    const Stats &stats() const { return stats_; }
    void reset_stats() { stats_ = Stats(); }
    const Config &config() const { return cfg_; }
    uint64_t arena_free() const { return arena_.free_bytes(); }
    // Offset of a request's outputs (valid from admission until release).
    bool output_offset(uint64_t ticket, uint64_t *off) const;

private:
    void retire(double now);
    void admit(double now);
    int launch(double now);

    Config cfg_;
    Executor *ex_;
    Arena arena_;
    uint64_t next_ticket_ = 1;
    std::deque<Request *> waiting_;   // arrived, not admitted (FIFO)
    std::deque<Request *> admitted_;  // outputs allocated, not launched
    std::vector<Batch> slots_;        // per slot, reqs empty = free
    std::deque<Request *> completed_;
    std::map<uint64_t, Request *> live_;  // ticket -> request (until release)
    Stats stats_;
};

// The scheduler as a service for many threads: one worker thread runs
// step() whenever it is not idle (and polls every 20 us when it is); any
// thread may submit, take completions, release outputs, read statistics or
// wait for the queue to drain.  Every access to the scheduler, and every call
// of the executor (from step()), happens under one mutex.  `clock` returns
// seconds on the service's clock; `on_start` runs first on the worker
// thread (the server binds its GPU there).
class Service {
public:
    Service(const Config &cfg, Executor *ex, std::function<double()> clock,
            std::function<void()> on_start = {});
    ~Service();  // stops the worker; drain first to finish queued work

    // t_arrival < 0: now.  Returns 0, -3 (larger than the budget) or -6 (full).
    int submit(Request r, uint64_t *ticket);
    std::vector<Request> take_completed(size_t max);
    // 0, -5 (still queued or running) or -1 (unknown ticket).
    int release(uint64_t ticket);
    // Waits until nothing is queued or running; false on timeout.
    bool drain(double timeout_s);
    // f(const Scheduler &) under the lock.
    template <typename F> auto inspect(F f) {
        std::lock_guard<std::mutex> lk(mu_);
        return f(static_cast<const Scheduler &>(sched_));
    }
    void reset_stats();
    double now() const { return clock_(); }
    void stop();

private:
    void loop(std::function<void()> on_start);

    Scheduler sched_;
    std::function<double()> clock_;
    std::mutex mu_;
    std::atomic<bool> stop_{false};
    std::thread worker_;
};

// Quantile of a sample (nearest rank, q in [0, 1]); 0 if empty.
double quantile(std::vector<double> v, double q);

}  // namespace sched
}  // namespace sne
