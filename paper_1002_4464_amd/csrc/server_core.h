// Request scheduling for the served sort stream: admission by a device-memory budget, continuous
// batching of small requests into segmented launches, and completion tracking.  Pure host C++
// (no HIP): the device work goes through the Executor interface, so the policy is testable on a
// machine without a GPU.
//
// Model.  Requests arrive with their keys (and values) already in device memory, owned by the
// caller.  The server owns a device arena of `budget` bytes from which every launch takes its
// workspace (and, for a batch, a staging copy of its members).  A launch is a "unit": one plain
// sort of one request (in place on the caller's buffers), or one segmented sort of a batch of
// requests packed into staging.  Units run on `lanes` independent device queues, one unit per
// lane at a time, so up to `lanes` units overlap on the device.  Each pass of the scheduler
//   1. reaps finished units (their requests become DONE, their arena blocks and lanes free up);
//   2. while a lane is free, takes the oldest queued request; if it is small (fits one
//      segmented batch) it gathers the other queued small requests of the same key layout, in
//      arrival order, into one batch; the unit is admitted if its memory fits the arena, else
//      the batch is halved until it fits or the oldest request waits (first come, first served:
//      nothing overtakes a request that is waiting for memory).
// Requests that arrive while units run simply queue and join the next unit formed when a lane
// frees: that is the continuous batching.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace dsort {
namespace srv {

inline uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over [0, size) with 256-byte granules; coalesces on free.
class Arena {
  public:
    explicit Arena(uint64_t size = 0) { reset(size); }
    void reset(uint64_t size) {
        size_ = size & ~uint64_t(255);
        free_.clear();
        live_.clear();
        used_ = peak_ = 0;
        if (size_) free_[0] = size_;
    }
    bool alloc(uint64_t bytes, uint64_t &off) {
        bytes = (std::max<uint64_t>(bytes, 1) + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            live_[off] = bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t off) {
        auto it = live_.find(off);
        if (it == live_.end()) return;
        uint64_t start = off, len = it->second;
        live_.erase(it);
        used_ -= len;
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && start + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    size_t free_blocks() const { return free_.size(); }
    uint64_t largest_free() const {
        uint64_t b = 0;
        for (auto &f : free_) b = std::max(b, f.second);
        return b;
    }

  private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
    std::unordered_map<uint64_t, uint64_t> live_;
};

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2 };

// Checks one submitted request: a known key type (1 uint32, 2 uint64, 3 float32), values
// flag 0 or 1, n within `max_items`, and for every n >= 1 key (and value) pointers that are
// non-null and naturally aligned.  A request of one item is still read and written in place by
// the batch staging copies, so n = 1 needs valid pointers too; only n = 0 may pass null.
inline bool request_valid(int key_type, int with_values, const void *keys, const void *vals,
                          uint64_t n, uint64_t max_items) {
    if (key_type != 1 && key_type != 2 && key_type != 3) return false;
    if (with_values != 0 && with_values != 1) return false;
    if (n > max_items) return false;
    if (n == 0) return true;
    if (!keys || (with_values && !vals)) return false;
    if (((uintptr_t)keys & (key_type == 2 ? 7u : 3u)) != 0) return false;
    if (with_values && ((uintptr_t)vals & 3u) != 0) return false;
    return true;
}

struct Request {
    uint64_t ticket = 0;
    int key_type = 0;
    bool values = false;
    void *keys = nullptr;
    uint32_t *vals = nullptr;
    uint64_t n = 0;
    int state = kQueued;  // or a negative status
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t unit = 0;    // unit that ran it
};

struct Unit {
    uint64_t id = 0;
    int lane = -1;
    int failed = 0;                        // launch status when the launch failed
    int key_type = 0;
    bool values = false;
    bool batched = false;
    std::vector<Request *> reqs;
    uint64_t total = 0, max_seg = 0;       // items, longest member
    uint64_t ws_off = 0, ws_bytes = 0;     // arena block: workspace (+ staging, + tables)
    void *token = nullptr;                 // executor's completion handle
};

// What the scheduler needs from the device side.  All byte counts are arena bytes.
class Executor {
  public:
    virtual ~Executor() {}
    virtual int lanes() const = 0;
    // Largest request a batch may hold (items) for a key layout; larger ones run alone.
    virtual uint64_t batch_item_limit(int key_type, bool values) const = 0;
    // Arena bytes of one unit (0 = impossible).
    virtual uint64_t unit_bytes(const Unit &u) const = 0;
    // Enqueue the unit on its lane; ws is the arena offset of its block.  Returns 0 or a
    // negative status (the unit's requests then fail with it).  A failed launch may have
    // enqueued part of the unit's work: poll() must still report the unit finished only once
    // nothing enqueued for it can touch its block or its requests' buffers any more.
    virtual int launch(Unit &u) = 0;
    // 1 finished, 0 still running, negative: failed with that status.
    virtual int poll(Unit &u) = 0;
    virtual void retire(Unit &) {}
    // Called once on the scheduler's background thread before its first pass.
    virtual void on_thread_start() {}
};

struct Stats {
    uint64_t submitted = 0, completed = 0, failed = 0;
    uint64_t units = 0, batched_units = 0, batched_requests = 0;
    uint64_t max_batch = 0, peak_arena = 0, peak_running = 0;
};

struct Limits {
    uint64_t max_batch_items = 1ull << 28;   // items per batched unit
    uint64_t max_batch_requests = 4096;      // requests per batched unit
};

class Scheduler {
  public:
    Scheduler(Executor *ex, uint64_t budget, uint32_t max_inflight, Limits lim = Limits{})
        : ex_(ex), max_inflight_(max_inflight ? max_inflight : 1u), lim_(lim) {
        arena_.reset(budget);
        lane_busy_.assign((size_t)ex_->lanes(), false);
    }

    // Validates against what could ever run; the request is queued (not yet admitted).
    int submit(const Request &r, uint64_t *ticket, int *why) {
        std::lock_guard<std::mutex> g(mu_);
        Unit probe;
        probe.key_type = r.key_type;
        probe.values = r.values;
        probe.reqs = {};
        probe.total = r.n;
        probe.max_seg = r.n;
        const uint64_t need = ex_->unit_bytes(probe);
        if (need == 0 || need > arena_.size()) {
            if (why) *why = 1;
            return -1;
        }
        Request *q = new Request(r);
        q->ticket = ++next_ticket_;
        q->state = kQueued;
        q->t_submit = now_ns();
        all_[q->ticket] = q;
        queue_.push_back(q);
        ++st_.submitted;
        *ticket = q->ticket;
        cv_.notify_all();
        return 0;
    }

    bool lookup(uint64_t ticket, Request &out) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = all_.find(ticket);
        if (it == all_.end()) return false;
        out = *it->second;
        return true;
    }

    // Forget a finished request (frees its record).  False if unknown or not finished.
    bool forget(uint64_t ticket) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = all_.find(ticket);
        if (it == all_.end() || it->second->state == kQueued || it->second->state == kRunning)
            return false;
        delete it->second;
        all_.erase(it);
        return true;
    }

    Stats stats() {
        std::lock_guard<std::mutex> g(mu_);
        Stats s = st_;
        s.peak_arena = arena_.peak();
        return s;
    }

    // One scheduling pass; returns true if anything changed.
    bool step() {
        std::lock_guard<std::mutex> g(mu_);
        return step_locked();
    }

    bool idle() {
        std::lock_guard<std::mutex> g(mu_);
        return queue_.empty() && running_.empty();
    }

    // Background loop: passes until stop(); sleeps briefly when nothing changed.
    void start() {
        run_ = true;
        th_ = std::thread([this] {
            ex_->on_thread_start();
            std::unique_lock<std::mutex> lk(mu_);
            while (run_) {
                bool changed = step_locked();
                if (!changed) {
                    // system_clock deadlines wait through pthread_cond_timedwait
                    const auto d = running_.empty() && queue_.empty()
                                       ? std::chrono::microseconds(5000)
                                       : std::chrono::microseconds(20);
                    cv_.wait_until(lk, std::chrono::system_clock::now() + d);
                }
            }
        });
    }

    void stop() {
        {
            std::lock_guard<std::mutex> g(mu_);
            run_ = false;
            cv_.notify_all();
        }
        if (th_.joinable()) th_.join();
    }

    // Runs passes on the calling thread until nothing is queued or running (for shutdown and
    // for tests without the background loop).  poll() must eventually report every unit.
    void drain() {
        while (true) {
            {
                std::lock_guard<std::mutex> g(mu_);
                step_locked();
                if (queue_.empty() && running_.empty()) return;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }

    ~Scheduler() {
        stop();
        for (auto &kv : all_) delete kv.second;
    }

    uint64_t arena_used() {
        std::lock_guard<std::mutex> g(mu_);
        return arena_.used();
    }

  private:
    bool small(const Request *r) const {
        return r->n <= ex_->batch_item_limit(r->key_type, r->values);
    }

    int free_lane() const {
        for (size_t i = 0; i < lane_busy_.size(); ++i)
            if (!lane_busy_[i]) return (int)i;
        return -1;
    }

    void finish(Unit *u, int status) {
        const uint64_t t = now_ns();
        for (Request *r : u->reqs) {
            r->state = status == 1 ? kDone : status;
            r->t_done = t;
            if (status == 1) ++st_.completed; else ++st_.failed;
            --inflight_;
        }
        arena_.release(u->ws_off);
        lane_busy_[(size_t)u->lane] = false;
        ex_->retire(*u);
    }

    bool step_locked() {
        bool changed = false;
        // 1. reap
        for (size_t i = 0; i < running_.size();) {
            Unit *u = running_[i];
            const int p = ex_->poll(*u);
            if (p == 0) {
                ++i;
                continue;
            }
            finish(u, u->failed ? u->failed : p);
            delete u;
            running_.erase(running_.begin() + (long)i);
            changed = true;
        }
        // 2. admit and launch
        while (!queue_.empty()) {
            const int lane = free_lane();
            if (lane < 0 || inflight_ >= max_inflight_) break;
            Request *head = queue_.front();
            Unit *u = new Unit;
            u->id = ++next_unit_;
            u->lane = lane;
            u->key_type = head->key_type;
            u->values = head->values;
            std::vector<size_t> picked{0};
            if (small(head)) {
                uint64_t items = head->n;
                const uint64_t room = max_inflight_ - inflight_;
                for (size_t q = 1; q < queue_.size() && picked.size() < room &&
                                   picked.size() < lim_.max_batch_requests;
                     ++q) {
                    const Request *r = queue_[q];
                    if (r->key_type != head->key_type || r->values != head->values || !small(r))
                        continue;
                    if (items + r->n > lim_.max_batch_items) continue;
                    items += r->n;
                    picked.push_back(q);
                }
            }
            // shrink until the unit's memory fits (the oldest request always stays in)
            uint64_t need = 0, off = 0;
            bool ok = false;
            while (true) {
                set_members(*u, picked);
                need = ex_->unit_bytes(*u);
                if (need && arena_.alloc(need, off)) {
                    ok = true;
                    break;
                }
                if (picked.size() == 1) break;
                picked.resize((picked.size() + 1) / 2);
            }
            if (!ok) {
                delete u;
                break;  // the oldest request waits for memory
            }
            u->ws_off = off;
            u->ws_bytes = need;
            const uint64_t t = now_ns();
            for (Request *r : u->reqs) {
                r->state = kRunning;
                r->t_admit = t;
                r->unit = u->id;
            }
            // remove picked requests from the queue (indices ascending)
            for (size_t k = picked.size(); k-- > 0;) queue_.erase(queue_.begin() + (long)picked[k]);
            inflight_ += (uint32_t)u->reqs.size();
            lane_busy_[(size_t)lane] = true;
            ++st_.units;
            if (u->batched) {
                ++st_.batched_units;
                st_.batched_requests += u->reqs.size();
                st_.max_batch = std::max<uint64_t>(st_.max_batch, u->reqs.size());
            }
            // A failed launch keeps its block and lane until poll() reports the lane drained:
            // work enqueued before the failure may still write them.
            u->failed = ex_->launch(*u);
            running_.push_back(u);
            st_.peak_running = std::max<uint64_t>(st_.peak_running, running_.size());
            changed = true;
        }
        return changed;
    }

    void set_members(Unit &u, const std::vector<size_t> &picked) {
        u.reqs.clear();
        u.total = 0;
        u.max_seg = 0;
        for (size_t k : picked) {
            Request *r = queue_[k];
            u.reqs.push_back(r);
            u.total += r->n;
            u.max_seg = std::max(u.max_seg, r->n);
        }
        u.batched = u.reqs.size() > 1;
    }

    Executor *ex_;
    uint32_t max_inflight_;
    Limits lim_;
    Arena arena_;
    std::vector<bool> lane_busy_;
    std::deque<Request *> queue_;
    std::vector<Unit *> running_;
    std::unordered_map<uint64_t, Request *> all_;
    uint64_t next_ticket_ = 0, next_unit_ = 0;
    uint32_t inflight_ = 0;
    Stats st_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread th_;
    bool run_ = false;
};

}  // namespace srv
}  // namespace dsort
