// Host-only tests of the served-stream scheduler (server_core.h) with a fake executor: the
// arena allocator against a byte-map model, admission by memory in arrival order, continuous
// batching, failure paths, and a multi-threaded stream.  Prints "OK <name>" per test; exits
// non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <random>
#include <set>
#include <vector>

#include "server_core.h"

using namespace dsort::srv;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

// Units finish when the test says so (or after `auto_polls` polls when > 0).
struct FakeExec : Executor {
    int nl = 2;
    uint64_t limit = 1000;       // batch item limit
    int auto_polls = 0;
    int fail_launch_on = -1;     // unit id whose launch fails
    int fail_poll_on = -1;       // unit id whose poll fails
    std::set<uint64_t> finished; // unit ids allowed to finish
    std::vector<std::vector<uint64_t>> launched;  // tickets per launched unit
    std::vector<int> polls;
    std::atomic<int> running{0};
    int max_running = 0;

    int lanes() const override { return nl; }
    uint64_t batch_item_limit(int, bool) const override { return limit; }
    uint64_t unit_bytes(const Unit &u) const override {
        return u.batched ? 1024 + u.total * 8 + u.reqs.size() * 16 : 512 + u.total * 4;
    }
    int launch(Unit &u) override {
        if (polls.size() <= u.id) polls.resize(u.id + 1, 0);
        if ((int)u.id == fail_launch_on) {
            // part of the unit's work was enqueued before the failure: it still occupies the
            // lane until poll() reports it drained
            ++running;
            return -4;
        }
        std::vector<uint64_t> t;
        for (auto *r : u.reqs) t.push_back(r->ticket);
        launched.push_back(t);
        int now = ++running;
        if (now > max_running) max_running = now;
        return 0;
    }
    int poll(Unit &u) override {
        if ((int)u.id == fail_poll_on) {
            --running;
            return -4;
        }
        int &p = polls[u.id];
        ++p;
        if (finished.count(u.id) || (auto_polls > 0 && p >= auto_polls)) {
            --running;
            return 1;
        }
        return 0;
    }
};

static Request req(uint64_t n, int kt = 1, bool v = false) {
    Request r;
    r.key_type = kt;
    r.values = v;
    r.n = n;
    return r;
}

static int state(Scheduler &s, uint64_t t) {
    Request r;
    CHECK(s.lookup(t, r));
    return r.state;
}

static void test_arena_model() {
    std::mt19937_64 rng(7);
    const uint64_t size = 1 << 20;
    Arena a(size);
    std::vector<uint8_t> used(size / 256, 0);
    std::vector<std::pair<uint64_t, uint64_t>> live;  // off, granules
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const uint64_t bytes = 1 + rng() % 20000;
            uint64_t off;
            const uint64_t g = (bytes + 255) / 256;
            // first fit in the model
            uint64_t run = 0, want = UINT64_MAX;
            for (uint64_t i = 0; i < used.size(); ++i) {
                run = used[i] ? 0 : run + 1;
                if (run == g) {
                    want = (i + 1 - g) * 256;
                    break;
                }
            }
            const bool ok = a.alloc(bytes, off);
            CHECK(ok == (want != UINT64_MAX));
            if (ok) {
                CHECK(off == want);
                for (uint64_t i = off / 256; i < off / 256 + g; ++i) {
                    CHECK(!used[i]);
                    used[i] = 1;
                }
                live.push_back({off, g});
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].first);
            for (uint64_t i = live[k].first / 256; i < live[k].first / 256 + live[k].second; ++i)
                used[i] = 0;
            live.erase(live.begin() + (long)k);
        }
        uint64_t u = 0;
        for (auto x : used) u += x;
        CHECK(a.used() == u * 256);
    }
    for (auto &l : live) a.release(l.first);
    CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == size);
    printf("OK arena_model\n");
}

static void test_batching_while_busy() {
    FakeExec ex;
    Scheduler s(&ex, 1 << 20, 64);
    uint64_t t[12];
    CHECK(s.submit(req(100), &t[0], nullptr) == 0);
    CHECK(s.submit(req(5000), &t[1], nullptr) == 0);  // large: alone
    s.step();
    CHECK(ex.launched.size() == 2);  // both lanes busy
    CHECK(ex.launched[0] == std::vector<uint64_t>{t[0]});
    for (int i = 2; i < 12; ++i) {
        // alternate layouts: u32 keys and u64 pairs
        CHECK(s.submit(i % 2 ? req(50 + i, 2, true) : req(50 + i), &t[i], nullptr) == 0);
    }
    s.step();
    CHECK(ex.launched.size() == 2);  // no lane free: everything waits
    CHECK(state(s, t[5]) == kQueued);
    ex.finished.insert(1);
    s.step();
    // lane 0 freed: the oldest waiting request (t[2], u32) and every queued u32 small one
    CHECK(state(s, t[0]) == kDone);
    CHECK(ex.launched.size() == 3);
    CHECK((ex.launched[2] == std::vector<uint64_t>{t[2], t[4], t[6], t[8], t[10]}));
    ex.finished.insert(2);
    s.step();
    CHECK((ex.launched[3] == std::vector<uint64_t>{t[3], t[5], t[7], t[9], t[11]}));
    ex.finished.insert(3);
    ex.finished.insert(4);
    s.step();
    s.step();
    for (int i = 0; i < 12; ++i) CHECK(state(s, t[i]) == kDone);
    Stats st = s.stats();
    CHECK(st.units == 4 && st.batched_units == 2 && st.batched_requests == 10);
    CHECK(st.max_batch == 5 && st.completed == 12);
    CHECK(s.arena_used() == 0);
    printf("OK batching_while_busy\n");
}

static void test_memory_order() {
    FakeExec ex;
    ex.nl = 4;
    // budget: a large request needs 512 + 4n bytes
    Scheduler s(&ex, 64 * 1024, 64);
    uint64_t a, b, c, d;
    CHECK(s.submit(req(9000), &a, nullptr) == 0);   // 36.5 KB
    CHECK(s.submit(req(8000), &b, nullptr) == 0);   // 32.5 KB: does not fit beside a
    CHECK(s.submit(req(10), &c, nullptr) == 0);     // tiny, but must not overtake b
    s.step();
    CHECK(ex.launched.size() == 1 && state(s, b) == kQueued && state(s, c) == kQueued);
    ex.finished.insert(1);
    s.step();
    CHECK(state(s, a) == kDone);
    CHECK(ex.launched.size() == 3);  // b, then c fits beside it
    CHECK(ex.launched[1] == std::vector<uint64_t>{b});
    CHECK(ex.launched[2] == std::vector<uint64_t>{c});
    // never admissible: rejected at submission
    int why = 0;
    CHECK(s.submit(req(100000), &d, &why) != 0 && why == 1);
    ex.auto_polls = 1;
    s.drain();
    CHECK(s.stats().peak_arena <= 64 * 1024);
    printf("OK memory_order\n");
}

static void test_batch_halves_to_fit() {
    FakeExec ex;
    ex.nl = 1;
    // batched bytes: 1024 + 8*total + 16*S.  Ten requests of 900 items: 73 KB > 40 KB budget
    Scheduler s(&ex, 40 * 1024, 64);
    std::vector<uint64_t> t(10);
    for (int i = 0; i < 10; ++i) CHECK(s.submit(req(900), &t[(size_t)i], nullptr) == 0);
    s.step();
    CHECK(ex.launched.size() == 1);
    CHECK(ex.launched[0].size() == 5);  // halved once: 1024 + 36000 + 80 bytes fits
    CHECK(ex.launched[0][0] == t[0]);
    ex.auto_polls = 1;
    s.drain();
    for (auto x : t) CHECK(state(s, x) == kDone);
    printf("OK batch_halves_to_fit\n");
}

static void test_inflight_cap() {
    FakeExec ex;
    ex.nl = 4;
    Scheduler s(&ex, 1 << 20, 3);
    std::vector<uint64_t> t(8);
    for (int i = 0; i < 8; ++i) CHECK(s.submit(req(2000 + i), &t[(size_t)i], nullptr) == 0);
    s.step();
    CHECK(ex.launched.size() == 3);  // three requests in flight at most
    ex.auto_polls = 1;
    s.drain();
    for (auto x : t) CHECK(state(s, x) == kDone);
    printf("OK inflight_cap\n");
}

// A failed launch keeps its arena block and lane until the executor reports the lane drained.
static void test_failed_launch_holds_block() {
    FakeExec ex;
    ex.nl = 1;
    ex.fail_launch_on = 1;
    Scheduler s(&ex, 1 << 20, 64);
    uint64_t a, b;
    CHECK(s.submit(req(5000), &a, nullptr) == 0);
    CHECK(s.submit(req(6000), &b, nullptr) == 0);
    s.step();
    CHECK(s.arena_used() > 0);       // unit 1 failed to launch but its block is still held
    CHECK(state(s, a) == kRunning);  // and its request is not reported yet
    CHECK(ex.launched.empty());      // the only lane is still taken: unit 2 waits
    s.step();
    CHECK(ex.launched.empty() && state(s, b) == kQueued);
    ex.finished.insert(1);           // the lane drains
    s.step();
    CHECK(state(s, a) == -4);
    CHECK(ex.launched.size() == 1 && state(s, b) == kRunning);
    ex.finished.insert(2);
    s.drain();
    CHECK(state(s, b) == kDone && s.arena_used() == 0);
    printf("OK failed_launch_holds_block\n");
}

// Submitted requests: every n >= 1 needs valid, aligned pointers (batch staging reads and writes
// even one-item requests); only n = 0 may pass null.
static void test_request_validation() {
    alignas(16) static uint64_t buf[4];
    char *p = (char *)buf;
    const uint64_t mx = 1ull << 32;
    CHECK(request_valid(1, 0, p, nullptr, 1, mx));
    CHECK(!request_valid(1, 0, nullptr, nullptr, 1, mx));
    CHECK(!request_valid(1, 1, p, nullptr, 1, mx));
    CHECK(!request_valid(2, 0, p + 4, nullptr, 1, mx));
    CHECK(!request_valid(1, 0, p + 2, nullptr, 5, mx));
    CHECK(!request_valid(1, 1, p, p + 1, 1, mx));
    CHECK(request_valid(2, 1, p, p + 4, 2, mx));
    CHECK(request_valid(3, 0, nullptr, nullptr, 0, mx));
    CHECK(!request_valid(4, 0, p, nullptr, 1, mx));
    CHECK(!request_valid(1, 2, p, p, 1, mx));
    CHECK(!request_valid(1, 0, p, nullptr, mx + 1, mx));
    printf("OK request_validation\n");
}

static void test_failures() {
    FakeExec ex;
    ex.fail_launch_on = 1;
    ex.fail_poll_on = 2;
    Scheduler s(&ex, 1 << 20, 64);
    uint64_t a, b, c;
    CHECK(s.submit(req(5000), &a, nullptr) == 0);
    CHECK(s.submit(req(6000), &b, nullptr) == 0);
    CHECK(s.submit(req(7000), &c, nullptr) == 0);
    ex.auto_polls = 1;
    s.drain();
    CHECK(state(s, a) == -4);
    CHECK(state(s, b) == -4);
    CHECK(state(s, c) == kDone);
    Stats st = s.stats();
    CHECK(st.failed == 2 && st.completed == 1);
    CHECK(s.arena_used() == 0);
    CHECK(s.forget(a) && !s.forget(a));
    Request r;
    CHECK(!s.lookup(a, r));
    printf("OK failures\n");
}

static void test_threaded_stream() {
    FakeExec ex;
    ex.nl = 3;
    ex.auto_polls = 3;
    Scheduler s(&ex, 1 << 22, 256);
    s.start();
    std::vector<std::thread> subs;
    std::vector<std::vector<uint64_t>> tickets(4);
    for (int k = 0; k < 4; ++k)
        subs.emplace_back([&, k] {
            std::mt19937 rng(k);
            for (int i = 0; i < 500; ++i) {
                uint64_t t;
                const uint64_t n = 1 + rng() % 3000;
                while (s.submit(req(n, 1 + (int)(rng() % 2)), &t, nullptr) != 0) {
                }
                tickets[(size_t)k].push_back(t);
                if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
            }
        });
    for (auto &th : subs) th.join();
    for (int spin = 0; spin < 20000 && !s.idle(); ++spin)
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    CHECK(s.idle());
    s.stop();
    std::set<uint64_t> seen;
    for (auto &v : ex.launched)
        for (auto t : v) CHECK(seen.insert(t).second);  // each request launched exactly once
    CHECK(seen.size() == 2000);
    for (auto &v : tickets)
        for (auto t : v) CHECK(state(s, t) == kDone);
    CHECK(ex.max_running <= 3);
    Stats st = s.stats();
    CHECK(st.completed == 2000 && st.batched_units > 0);
    printf("OK threaded_stream units=%llu batched=%llu max_batch=%llu\n",
           (unsigned long long)st.units, (unsigned long long)st.batched_units,
           (unsigned long long)st.max_batch);
}

int main() {
    test_arena_model();
    test_batching_while_busy();
    test_memory_order();
    test_batch_halves_to_fit();
    test_inflight_cap();
    test_failures();
    test_failed_launch_holds_block();
    test_request_validation();
    test_threaded_stream();
    printf("ALL OK\n");
    return 0;
}
