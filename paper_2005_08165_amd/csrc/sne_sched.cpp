// sne_sched.cpp - continuous-batching scheduler core (see sne_sched.h).
#include "sne_sched.h"

#include <algorithm>
#include <chrono>
#include <cmath>

namespace sne {
namespace sched {

Arena::Arena(uint64_t size, uint64_t align) : size_(size), align_(align ? align : 1), free_(size) {
    if (size_) holes_[0] = size_;
}

bool Arena::alloc(uint64_t bytes, uint64_t *offset) {
    bytes = round(bytes);
    for (auto it = holes_.begin(); it != holes_.end(); ++it) {
        if (it->second >= bytes) {
            const uint64_t off = it->first, len = it->second;
            holes_.erase(it);
            if (len > bytes) holes_[off + bytes] = len - bytes;
            free_ -= bytes;
            *offset = off;
            return true;
        }
    }
    return false;
}

void Arena::release(uint64_t offset, uint64_t bytes) {
    bytes = round(bytes);
    auto next = holes_.lower_bound(offset);
    uint64_t off = offset, len = bytes;
    if (next != holes_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            holes_.erase(prev);
        }
    }
    if (next != holes_.end() && off + len == next->first) {
        len += next->second;
        holes_.erase(next);
    }
    holes_[off] = len;
    free_ += bytes;
}

namespace {
constexpr double kHistLo = 1e-7;     // seconds: lower edge of bin 0
constexpr double kHistRatio = 1.01;  // upper / lower edge of a bin
constexpr int kHistBins = 2546;      // up to 1e-7 * 1.01^2546 > 1e4 s
}  // namespace

LatencyHistogram::LatencyHistogram() : bins_(kHistBins, 0) {}

void LatencyHistogram::add(double s) {
    if (!(s >= 0.0)) s = 0.0;
    int b = s <= kHistLo ? 0 : (int)(std::log(s / kHistLo) / std::log(kHistRatio));
    b = std::min(std::max(b, 0), kHistBins - 1);
    ++bins_[b];
    if (n_ == 0 || s < min_) min_ = s;
    if (n_ == 0 || s > max_) max_ = s;
    ++n_;
}

double LatencyHistogram::quantile(double q) const {
    if (n_ == 0) return 0.0;
    // the same rank rule as quantile(vector): index floor(q n), at most n - 1
    uint64_t k = (uint64_t)(q * (double)n_);
    if (k >= n_) k = n_ - 1;
    if (k == 0) return min_;
    if (k == n_ - 1) return max_;
    uint64_t seen = 0;
    for (int b = 0; b < kHistBins; ++b) {
        seen += bins_[b];
        if (seen > k) {
            const double hi = kHistLo * std::pow(kHistRatio, b + 1);
            return std::min(std::max(hi, min_), max_);
        }
    }
    return max_;
}

Scheduler::Scheduler(const Config &cfg, Executor *ex)
    : cfg_(cfg), ex_(ex), arena_(cfg.budget_bytes, cfg.align), slots_(cfg.max_inflight) {
    for (int i = 0; i < cfg_.max_inflight; ++i) slots_[i].slot = i;
}

Scheduler::~Scheduler() {
    for (auto &kv : live_) delete kv.second;
}

int Scheduler::inflight() const {
    int n = 0;
    for (const auto &b : slots_) n += b.reqs.empty() ? 0 : 1;
    return n;
}

int Scheduler::submit(const Request &r, uint64_t *ticket) {
    if (arena_.round(r.out_bytes) > arena_.size()) {
        ++stats_.rejected_budget;
        return -3;
    }
    if (waiting_.size() + admitted_.size() >= cfg_.queue_capacity) {
        ++stats_.rejected_full;
        return -6;
    }
    Request *q = new Request(r);
    q->ticket = next_ticket_++;
    if (stats_.submitted == 0) stats_.first_arrival = q->t_arrival;
    ++stats_.submitted;
    live_[q->ticket] = q;
    waiting_.push_back(q);
    if (ticket) *ticket = q->ticket;
    return 0;
}

void Scheduler::retire(double now) {
    for (auto &b : slots_) {
        if (b.reqs.empty() || !ex_->done(b)) continue;
        const int rc = ex_->result(b);
        for (Request *q : b.reqs) {
            q->t_done = now;
            q->status = rc;
            q->finished = true;
            if (rc == 0) {
                ++stats_.completed;
                stats_.pixels_done += (uint64_t)q->H * q->W;
                stats_.latency.add(q->t_done - q->t_arrival);
            } else {
                ++stats_.failed;
            }
            stats_.last_done = now;
            completed_.push_back(q);
        }
        b.reqs.clear();
        b.pixels = 0;
    }
}

void Scheduler::admit(double now) {
    // FIFO: the head waits for memory instead of being overtaken
    while (!waiting_.empty()) {
        Request *q = waiting_.front();
        uint64_t off = 0;
        if (!arena_.alloc(q->out_bytes, &off)) break;
        q->out_offset = off;
        q->has_output = true;
        q->t_admit = now;
        waiting_.pop_front();
        admitted_.push_back(q);
    }
}

int Scheduler::launch(double now) {
    int launched = 0;
    for (auto &b : slots_) {
        if (admitted_.empty()) break;
        if (!b.reqs.empty()) continue;
        uint64_t px = 0;
        while (!admitted_.empty() && (int)b.reqs.size() < cfg_.max_batch_frames) {
            Request *q = admitted_.front();
            const uint64_t p = (uint64_t)q->H * q->W;
            if (!b.reqs.empty() && px + p > cfg_.max_batch_pixels) break;
            px += p;
            q->t_launch = now;
            b.reqs.push_back(q);
            admitted_.pop_front();
        }
        b.pixels = px;
        const int rc = ex_->launch(b);
        ++stats_.batches;
        stats_.frames_in_batches += b.reqs.size();
        if (rc != 0) {
            // a failed launch fails its requests; the loop carries on
            for (Request *q : b.reqs) {
                q->status = rc;
                q->t_done = now;
                q->finished = true;
                ++stats_.failed;
                completed_.push_back(q);
            }
            b.reqs.clear();
            b.pixels = 0;
            continue;
        }
        ++launched;
    }
    return launched;
}

int Scheduler::step(double now) {
    retire(now);
    admit(now);
    return launch(now);
}

std::vector<Request> Scheduler::take_completed(size_t max) {
    std::vector<Request> out;
    while (!completed_.empty() && out.size() < max) {
        out.push_back(*completed_.front());
        completed_.pop_front();
    }
    return out;
}

int Scheduler::release(uint64_t ticket) {
    auto it = live_.find(ticket);
    if (it == live_.end()) return -1;
    Request *q = it->second;
    if (!q->finished) return -5;  // still queued or running
    if (q->has_output) arena_.release(q->out_offset, q->out_bytes);
    // drop from the completed queue if the client never took it
    for (auto c = completed_.begin(); c != completed_.end(); ++c)
        if (*c == q) {
            completed_.erase(c);
            break;
        }
    live_.erase(it);
    delete q;
    return 0;
}

bool Scheduler::output_offset(uint64_t ticket, uint64_t *off) const {
    auto it = live_.find(ticket);
    if (it == live_.end()) return false;
    *off = it->second->out_offset;
    return true;
}

Service::Service(const Config &cfg, Executor *ex, std::function<double()> clock,
                 std::function<void()> on_start)
    : sched_(cfg, ex), clock_(std::move(clock)) {
    worker_ = std::thread(&Service::loop, this, std::move(on_start));
}

Service::~Service() { stop(); }

void Service::stop() {
    stop_.store(true, std::memory_order_relaxed);
    if (worker_.joinable()) worker_.join();
}

void Service::loop(std::function<void()> on_start) {
    if (on_start) on_start();
    while (!stop_.load(std::memory_order_relaxed)) {
        bool busy;
        {
            std::lock_guard<std::mutex> lk(mu_);
            sched_.step(clock_());
            busy = !sched_.idle();
        }
        if (busy)
            std::this_thread::yield();
        else
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

int Service::submit(Request r, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    if (r.t_arrival < 0) r.t_arrival = clock_();
    return sched_.submit(r, ticket);
}

std::vector<Request> Service::take_completed(size_t max) {
    std::lock_guard<std::mutex> lk(mu_);
    return sched_.take_completed(max);
}

int Service::release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    return sched_.release(ticket);
}

bool Service::drain(double timeout_s) {
    const auto t_end =
        std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (sched_.idle()) return true;
        }
        if (std::chrono::steady_clock::now() > t_end) return false;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

void Service::reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    sched_.reset_stats();
}

double quantile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t i = (size_t)(q * (double)v.size());
    if (i >= v.size()) i = v.size() - 1;
    return v[i];
}

}  // namespace sched
}  // namespace sne
