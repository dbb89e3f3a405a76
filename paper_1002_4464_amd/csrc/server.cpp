// Served sort stream: the device side of the scheduler in server_core.h and its C ABI.
//
// A server owns one device arena of the HBM budget, `lanes` HIP streams of default priority with
// one completion event each, and per lane pinned host memory for batch descriptors and for the
// unit's kernel status word (read back with the unit; a non-zero word fails its requests).  A launch
// is admitted when its requests' data plus its workspace fit what is left of the budget; the
// workspace part is carved from the arena (the data part is reserved there too, unused, so one
// allocator keeps the account).  A plain
// unit runs Algorithm 1 in place on the request's buffers with a workspace block from the arena.
// A batched unit (several small requests of one key layout) copies its members into a staging
// block, runs one segmented sort over them (each request one segment), and copies the results
// back, all on its lane's stream.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "dsort.h"
#include "dsort_internal.h"
#include "server_core.h"

namespace dsort {
namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

uint32_t key_bytes_of(int kt) { return kt == DSORT_U64 ? 8u : 4u; }

class HipExecutor : public srv::Executor {
  public:
    int init(int device, uint32_t lanes, uint64_t budget, uint32_t max_batch_requests) {
        device_ = device;
        max_req_ = max_batch_requests;
        if (hipSetDevice(device) != hipSuccess) return DSORT_E_HIP;
        if (hipMalloc(&arena_, budget) != hipSuccess) {
            arena_ = nullptr;
            (void)hipGetLastError();
            return DSORT_E_NOMEM;
        }
        table_bytes_ = al256((size_t)max_req_ * 16 + ((size_t)max_req_ + 1) * 8);
        for (uint32_t i = 0; i < lanes; ++i) {
            hipStream_t s;
            hipEvent_t e;
            void *h = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return DSORT_E_HIP;
            streams_.push_back(s);
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return DSORT_E_HIP;
            events_.push_back(e);
            // the batch descriptor table, then one word for the unit's kernel status flags
            if (hipHostMalloc(&h, table_bytes_ + 256, hipHostMallocDefault) != hipSuccess)
                return DSORT_E_HIP;
            pinned_.push_back(h);
        }
        return DSORT_OK;
    }

    ~HipExecutor() override {
        for (hipStream_t s : streams_) (void)hipStreamSynchronize(s);
        for (hipEvent_t e : events_) (void)hipEventDestroy(e);
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        for (void *h : pinned_) (void)hipHostFree(h);
        if (arena_) (void)hipFree(arena_);
    }

    int lanes() const override { return (int)streams_.size(); }

    uint64_t batch_item_limit(int key_type, bool values) const override {
        return seg_limit(key_type, values);
    }

    // Budget bytes of a unit: the requests' own data (counted, not allocated: it lives in the
    // callers' buffers) plus the arena block it takes.  Arena block: plain = the sort's
    // workspace; batched = segmented workspace, then staging keys, staging values, the request
    // pointer tables and the offsets.
    uint64_t unit_bytes(const srv::Unit &u) const override {
        const uint64_t data = u.total * (key_bytes_of(u.key_type) + (u.values ? 4u : 0u));
        const uint64_t blk = block_bytes(u);
        return blk ? data + blk : 0;
    }

    uint64_t block_bytes(const srv::Unit &u) const {
        if (!u.batched) {
            if (u.total <= 1) return 256;
            Geom g;
            if (make_geom(u.key_type, u.values, u.total, dsort_tuning_t{}, g) != DSORT_OK)
                return 0;
            return al256(g.total);
        }
        const uint64_t S = u.reqs.size();
        if (S > max_req_) return 0;
        SegGeom sg;
        if (make_seg_geom(u.key_type, u.values, u.total, S, u.max_seg, SegTuning{}, sg) != DSORT_OK) return 0;
        size_t b = al256(sg.total);
        b += al256(u.total * key_bytes_of(u.key_type));
        if (u.values) b += al256(u.total * 4);
        b += table_bytes_;
        return b;
    }

    int launch(srv::Unit &u) override {
        const size_t lane = (size_t)u.lane;
        hipStream_t st = streams_[lane];
        char *blk = (char *)arena_ + u.ws_off;
        // The lane's previous unit has finished (its lane was free), so its status word is
        // no longer being written.
        uint32_t *status = lane_status(lane);
        *status = 0;
        const int rc = enqueue(u, st, blk);
        // The unit's status flags (the first word of its workspace block) come back with the
        // unit; poll() fails the unit if a kernel raised any.
        if (rc == DSORT_OK && ran_pipeline(u) &&
            hipMemcpyAsync(status, blk, 4, hipMemcpyDeviceToHost, st) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(st);
            return DSORT_E_HIP;
        }
        // Recorded after a failure too: whatever was enqueued before it must have finished
        // before poll() lets the scheduler hand the block and the lane to another unit.
        if (hipEventRecord(events_[lane], st) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(st);
            (void)hipEventSynchronize(events_[lane]);
            return rc != DSORT_OK ? rc : DSORT_E_HIP;
        }
        return rc;
    }

    int poll(srv::Unit &u) override {
        const hipError_t e = hipEventQuery(events_[(size_t)u.lane]);
        if (e == hipErrorNotReady) return 0;
        if (e != hipSuccess) {
            set_last_error("server", hipGetErrorName(e), hipGetErrorString(e));
            return DSORT_E_HIP;
        }
        const uint32_t flags = *lane_status((size_t)u.lane);
        if (flags != 0) {
            char buf[64];
            snprintf(buf, sizeof buf, "kernel status flags 0x%x", flags);
            set_last_error("server", "unit failed", buf);
            return DSORT_E_HIP;
        }
        return 1;
    }

    void on_thread_start() override { (void)hipSetDevice(device_); }

  private:
    uint32_t *lane_status(size_t lane) const {
        return (uint32_t *)((char *)pinned_[lane] + table_bytes_);
    }

    static bool ran_pipeline(const srv::Unit &u) { return u.batched || u.reqs[0]->n > 1; }

    // Enqueues the unit's work on st; returns the first failure (work enqueued before it stays
    // enqueued).
    int enqueue(srv::Unit &u, hipStream_t st, char *blk) {
        const size_t lane = (size_t)u.lane;
        if (!u.batched) {
            srv::Request *r = u.reqs[0];
            if (r->n <= 1) return DSORT_OK;
            Geom g;
            const int rc = make_geom(r->key_type, r->values, r->n, dsort_tuning_t{}, g);
            return rc == DSORT_OK ? run_pipeline(g, r->keys, r->vals, blk, st, nullptr) : rc;
        }
        const uint32_t S = (uint32_t)u.reqs.size();
        SegGeom sg;
        int rc = make_seg_geom(u.key_type, u.values, u.total, S, u.max_seg, SegTuning{}, sg);
        if (rc != DSORT_OK) return rc;
        char *p = blk + al256(sg.total);
        void *stage_keys = p;
        p += al256(u.total * key_bytes_of(u.key_type));
        uint32_t *stage_vals = nullptr;
        if (u.values) {
            stage_vals = (uint32_t *)p;
            p += al256(u.total * 4);
        }
        char *dev_tab = p;
        // descriptor table: S key pointers, S value pointers, S + 1 offsets
        uint64_t *h = (uint64_t *)pinned_[lane];
        uint64_t pos = 0;
        for (uint32_t i = 0; i < S; ++i) {
            const srv::Request *r = u.reqs[i];
            h[i] = (uint64_t)(uintptr_t)r->keys;
            h[S + i] = (uint64_t)(uintptr_t)r->vals;
            h[2 * S + i] = pos;
            pos += r->n;
        }
        h[3 * S] = pos;
        const size_t tb = ((size_t)3 * S + 1) * 8;
        if (hipMemcpyAsync(dev_tab, h, tb, hipMemcpyHostToDevice, st) != hipSuccess) {
            set_last_error("batch table", "hipMemcpyAsync", "failed");
            (void)hipGetLastError();
            return DSORT_E_HIP;
        }
        const uint64_t *d_keysp = (const uint64_t *)dev_tab;
        const uint64_t *d_valsp = d_keysp + S;
        const uint64_t *d_off = d_keysp + 2 * S;
        const int kb = (int)key_bytes_of(u.key_type);
        rc = launch_pack(kb, d_keysp, d_valsp, d_off, S, u.total, stage_keys, stage_vals, false,
                         st);
        if (rc == DSORT_OK) rc = run_segmented(sg, stage_keys, stage_vals, d_off, blk, st, nullptr);
        if (rc == DSORT_OK)
            rc = launch_pack(kb, d_keysp, d_valsp, d_off, S, u.total, stage_keys, stage_vals,
                             true, st);
        return rc;
    }

    int device_ = 0;
    uint32_t max_req_ = 0;
    void *arena_ = nullptr;
    size_t table_bytes_ = 0;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> events_;
    std::vector<void *> pinned_;
};

}  // namespace
}  // namespace dsort

struct dsort_server_s {
    uint32_t magic;
    dsort::HipExecutor *ex;
    dsort::srv::Scheduler *sched;
};

static constexpr uint32_t kServerMagic = 0x44535256u;  // "DSRV"

static bool server_ok(const dsort_server_s *s) { return s && s->magic == kServerMagic; }

extern "C" {

int dsort_server_create(dsort_server_t *out, uint64_t hbm_budget_bytes, uint32_t max_inflight,
                        uint32_t lanes) {
    if (!out) return DSORT_E_INVALID;
    *out = nullptr;
    if (hbm_budget_bytes < (1u << 20) || lanes == 0 || lanes > 16 || max_inflight == 0)
        return DSORT_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DSORT_E_HIP;
    dsort::srv::Limits lim;
    lim.max_batch_requests = max_inflight < 4096 ? max_inflight : 4096;
    auto *ex = new (std::nothrow) dsort::HipExecutor();
    if (!ex) return DSORT_E_NOMEM;
    int rc = ex->init(dev, lanes, hbm_budget_bytes, (uint32_t)lim.max_batch_requests);
    if (rc != DSORT_OK) {
        delete ex;
        return rc;
    }
    auto *sched = new (std::nothrow) dsort::srv::Scheduler(ex, hbm_budget_bytes, max_inflight, lim);
    auto *s = new (std::nothrow) dsort_server_s{kServerMagic, ex, sched};
    if (!sched || !s) {
        delete sched;
        delete s;
        delete ex;
        return DSORT_E_NOMEM;
    }
    sched->start();
    *out = s;
    return DSORT_OK;
}

int dsort_submit(dsort_server_t srv, const dsort_request_t *req, uint64_t *ticket) {
    if (!server_ok(srv) || !req || !ticket) return DSORT_E_INVALID;
    const int kt = req->key_type;
    if (!dsort::srv::request_valid(kt, req->with_values, req->d_keys, req->d_values, req->n,
                                   dsort::kMaxItems))
        return DSORT_E_INVALID;
    dsort::srv::Request r;
    r.key_type = kt;
    r.values = req->with_values != 0;
    r.keys = req->d_keys;
    r.vals = req->with_values ? req->d_values : nullptr;
    r.n = req->n;
    int why = 0;
    if (srv->sched->submit(r, ticket, &why) != 0) return DSORT_E_CAPACITY;
    return DSORT_OK;
}

int dsort_poll(dsort_server_t srv, uint64_t ticket, dsort_result_t *out) {
    if (!server_ok(srv) || !out) return DSORT_E_INVALID;
    dsort::srv::Request r;
    if (!srv->sched->lookup(ticket, r)) return DSORT_E_TICKET;
    memset(out, 0, sizeof(*out));
    out->state = r.state;
    out->t_submit_ns = r.t_submit;
    out->t_admit_ns = r.t_admit;
    out->t_done_ns = r.t_done;
    out->unit = r.unit;
    return DSORT_OK;
}

int dsort_release(dsort_server_t srv, uint64_t ticket) {
    if (!server_ok(srv)) return DSORT_E_INVALID;
    dsort::srv::Request r;
    if (!srv->sched->lookup(ticket, r)) return DSORT_E_TICKET;
    if (r.state == dsort::srv::kQueued || r.state == dsort::srv::kRunning) return DSORT_E_INVALID;
    return srv->sched->forget(ticket) ? DSORT_OK : DSORT_E_TICKET;
}

int dsort_server_stats(dsort_server_t srv, dsort_server_stats_t *out) {
    if (!server_ok(srv) || !out) return DSORT_E_INVALID;
    const dsort::srv::Stats s = srv->sched->stats();
    memset(out, 0, sizeof(*out));
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->failed = s.failed;
    out->units = s.units;
    out->batched_units = s.batched_units;
    out->batched_requests = s.batched_requests;
    out->max_batch = s.max_batch;
    out->peak_arena_bytes = s.peak_arena;
    out->peak_running_units = s.peak_running;
    return DSORT_OK;
}

int dsort_server_destroy(dsort_server_t srv) {
    if (!srv) return DSORT_OK;
    if (!server_ok(srv)) return DSORT_E_INVALID;
    srv->sched->stop();
    srv->sched->drain();
    srv->magic = 0;
    delete srv->sched;
    delete srv->ex;
    delete srv;
    return DSORT_OK;
}

}  // extern "C"
