// The pipeline of Algorithm 1 of Dehne & Zaboli, "Deterministic Sample Sort For GPUs"
// (Section 4), for gfx950 (CDNA4, wave64): the host code that enqueues the kernels of steps.h
// (built from the device primitives of sort_primitives.h), and the staging kernel of served
// batches.
//
// Stages (one kernel each unless noted):
//   k_tile<MODE_SAMPLE>   Steps 1-3: load one sublist of L items, sort it in LDS, write it
//                         back sorted, emit its s equidistant samples (positions kw-1).
//   k_sort_samples /      Step 4: sort the m*s samples -- one workgroup per segment when they
//   k_merge_round         fit in LDS, else workgroup chunk sorts plus global merge rounds.
//   k_rank                Steps 5-6: read global sample g_j = S[jm-1], locate it in every
//                         sorted sublist, write a_ij.
//   k_scan_*              Step 7: bucket-major exclusive prefix sum of the m x s matrix
//                         (column sums, scan of the column sums, update of every column).
//   k_tile<GIN>           Step 8 of a first level fused into Steps 1-3 of the second: each
//                         second-level sublist is gathered from the first level's pieces.
//   k_gather_bsort        Steps 8-9 fused: one workgroup per bucket gathers its pieces into LDS
//                         and sorts them (one launch per bucket size class).
//   k_tile<MODE_FINAL>    the whole input when it fits one workgroup.
//   k_seg_prepare         set-up of a batch of independent sorts (segmented sort).
//   k_pack                copies between requests' buffers and a batch's staging array.
// For inputs where one level would need too many samples, Step 9 runs Algorithm 1 again on
// every bucket (the buckets become the segments of a second level).
//
// Order: items compare under the total order (key, sublist i, sorted rank r); samples are the
// composites (key, i*L + r).  float32 keys are mapped to their IEEE totalOrder image on the
// first load and back on the last store, so every intermediate holds unsigned order keys.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <vector>

#include "dsort_internal.h"
#include "sort_primitives.h"
#include "steps.h"

namespace dsort {
namespace {

// ------------------------------------------------------------------------------ host driver

#define DS_CHECK_LAUNCH()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return DSORT_E_HIP; \
    } while (0)

// Launch with optional timing events around it; a failed launch is recorded for
// dsort_last_error() with the stage name and the HIP error.
#define DS_LAUNCH(NAME, KERNEL, GRID, BLOCK, ...)                                   \
    do {                                                                            \
        void *ev1_ = nullptr;                                                       \
        if (tm && stage_begin(*tm, NAME, st, &ev1_) != DSORT_OK)                    \
            return record_error(NAME, hipGetLastError());                           \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, st, __VA_ARGS__);                \
        {                                                                           \
            const hipError_t e_ = hipGetLastError();                                \
            if (e_ != hipSuccess) return record_error(NAME, e_);                    \
        }                                                                           \
        if (ev1_ && hipEventRecord((hipEvent_t)ev1_, st) != hipSuccess)             \
            return record_error(NAME, hipGetLastError());                           \
    } while (0)

int record_error(const char *stage, hipError_t e) {
    set_last_error(stage, hipGetErrorName(e), hipGetErrorString(e));
    return DSORT_E_HIP;
}

void *pool_event(Timing &t) {
    if (t.used == t.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        t.pool.push_back((void *)e);
    }
    return t.pool[t.used++];
}

int stage_begin(Timing &t, const char *name, hipStream_t st, void **ev1) {
    void *a = pool_event(t);
    void *b = pool_event(t);
    if (!a || !b) return DSORT_E_HIP;
    if (hipEventRecord((hipEvent_t)a, st) != hipSuccess) return DSORT_E_HIP;
    t.recs.push_back(StageRec{name, a, b});
    *ev1 = b;
    return DSORT_OK;
}

// Size classes of the fused Steps 8-9 per LDS element type (ascending; the last is the bucket
// capacity of the plan).
template <class T> struct ClassCaps;
template <> struct ClassCaps<uint32_t> {
    static constexpr uint32_t n = 8;
    static constexpr uint32_t cap[8] = {2048, 4096, 6144, 8192, 10240, 12288, 16384, 32768};
};
template <> struct ClassCaps<uint64_t> {
    static constexpr uint32_t n = 7;
    static constexpr uint32_t cap[8] = {2048, 4096, 6144, 8192, 10240, 12288, 16384, 0};
};
template <> struct ClassCaps<C128> {
    static constexpr uint32_t n = 5;
    static constexpr uint32_t cap[8] = {1024, 2048, 4096, 6144, 8192, 0, 0, 0};
};

constexpr uint32_t kNumCUs = 256;
constexpr uint32_t kListedGrid = 1024;  // workgroups of the listed-bucket copies

// Side streams on which the bucket size classes of one call run side by side, so that the
// single-bucket latency of a sparsely used class and the tail of a busy one overlap other
// classes' work; the call's stream waits for all of them before its next launch.  One set per
// device for the process (default priority, non-blocking), created on the first call that is
// not being captured; a call's fork and join are enqueued under one lock, so that calls from
// several host threads never interleave their event records.
constexpr int kForkStreams = 3;
struct ForkSet {
    hipStream_t side[kForkStreams];
    hipEvent_t fork;
    hipEvent_t join[kForkStreams];
};
std::mutex g_fork_mu;

// The device's set (nullptr if it cannot be made now); the caller holds g_fork_mu.
ForkSet *fork_set(hipStream_t st) {
    static std::map<int, ForkSet> sets;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = sets.find(dev);
    if (it != sets.end()) return &it->second;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return nullptr;
    ForkSet f{};
    bool ok = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kForkStreams && ok; ++i)
        ok = hipStreamCreateWithFlags(&f.side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return nullptr;  // partly made objects are left alone; the call runs on one stream
    }
    return &sets.emplace(dev, f).first->second;
}

// Workgroups of `kernel` (blocks of `block` threads, static LDS only) that the current device
// holds at once, from the runtime's occupancy calculator; `fallback` when it cannot say.
template <class F> uint32_t resident_blocks(F kernel, uint32_t block, uint32_t fallback) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)block, 0) !=
            hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        (void)hipGetLastError();  // not a launch failure: keep it out of the next check
        return fallback;
    }
    return (uint32_t)cus * (uint32_t)per_cu;
}

template <class K, bool V, bool F32> struct Pipeline {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    static constexpr int TE = (sizeof(typename R::T) >= 16) ? 8 : 16;  // Step 2 items/thread
    static constexpr int TCAP = TE * 1024;                            // largest L
    static constexpr int FE = (!V && sizeof(K) == 4) ? 32 : TE;       // Step 9 items/thread
    static constexpr int FCAP = FE * 1024;                            // bucket capacity
    static constexpr int SE = sizeof(SC) >= 16 ? 8 : 16;
    static constexpr int SCAP = SE * 1024;
    static constexpr int ME = SE / 2;  // merge rounds: half the tile, two workgroups per CU
    static constexpr int MCAP = ME * 1024;
    using T = typename R::T;
    using CC = ClassCaps<T>;
    static_assert(CC::cap[CC::n - 1] == (uint32_t)FCAP, "last class must be the bucket capacity");

    static Classes classes(uint32_t *status, uint32_t *lists, uint32_t stride) {
        Classes c{};
        c.n = CC::n;
        for (uint32_t i = 0; i < CC::n; ++i) c.cap[i] = CC::cap[i];
        c.count = status + 1;
        c.list = lists;
        c.stride = stride;
        return c;
    }

    // One persistent launch per size class, each exactly as large as the device can hold at
    // once (the runtime's occupancy figure, which counts registers as well as LDS and wave
    // slots: a grid beyond it would run its surplus as a second, serial round).  Class I goes
    // to stream cs[I].
    template <uint32_t I, bool XIN = false>
    static int gather_classes(const GatherArgs &a, const hipStream_t *cs, Timing *tm) {
        if constexpr (I < CC::n) {
            hipStream_t st = cs[I];
            constexpr int CAP = (int)CC::cap[I];
            constexpr int GE = GatherE<K, V, CAP>::E;
            constexpr uint32_t GBD = CAP / GE;
            constexpr uint32_t glds = (lds_elems<T>(CAP) + 1) * sizeof(T) + 8 * (kMaxPieces + 1);
            constexpr uint32_t gby_lds = 163840u / glds;
            constexpr uint32_t gby_waves = 32u / ((GBD + 63) / 64);
            constexpr uint32_t gocc = gby_lds < gby_waves ? gby_lds : gby_waves;
            static const uint32_t slots = resident_blocks(k_gather_bsort<K, V, CAP, F32, XIN>,
                                                          GBD, kNumCUs * (gocc ? gocc : 1u));
            const uint32_t grid = min(a.stride, slots);
            DS_LAUNCH("s89_gather_sort", (k_gather_bsort<K, V, CAP, F32, XIN>), dim3(grid),
                      dim3(GBD), a, I);
            return gather_classes<I + 1, XIN>(a, cs, tm);
        }
        return DSORT_OK;
    }

    // The fused Steps 8-9 of one level: every size class one after another on st, or, when
    // `fork` (and no per-kernel timing is asked for), class i on stream i mod 4 of st and the
    // three side streams.  Segmented sorts fork: their buckets spread over all classes, and
    // side by side the sparsely used classes fill the busy ones' tails.  Plain sorts do not:
    // their buckets crowd into two neighbouring classes, whose persistent grids side by side
    // only contend for the same CUs (measured slower).
    // With join == false the side streams are left running and *forked tells whether there
    // are any: the caller must join_side(st) before work on st that depends on them (and
    // before returning, failed launches included).
    template <bool XIN = false>
    static int launch_classes(const GatherArgs &a, hipStream_t st, Timing *tm, bool fork,
                              bool join = true, bool *forked = nullptr) {
        hipStream_t cs[kMaxClasses];
        for (auto &c : cs) c = st;
        if (forked) *forked = false;
        if (!fork || tm) return gather_classes<0, XIN>(a, cs, tm);
        // A call being captured into a graph stays on its own stream: forking would pull the
        // shared side streams into the capture, where other threads' calls enqueue too.
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            return gather_classes<0, XIN>(a, cs, tm);
        }
        int rc;
        {
            std::lock_guard<std::mutex> lock(g_fork_mu);
            ForkSet *fs = fork_set(st);
            if (!fs) return gather_classes<0, XIN>(a, cs, tm);
            for (uint32_t i = 0; i < (uint32_t)kMaxClasses; ++i)
                if (i % (1 + kForkStreams)) cs[i] = fs->side[i % (1 + kForkStreams) - 1];
            if (hipEventRecord(fs->fork, st) != hipSuccess)
                return record_error("s89_fork", hipGetLastError());
            for (int i = 0; i < kForkStreams; ++i)
                if (hipStreamWaitEvent(fs->side[i], fs->fork, 0) != hipSuccess)
                    return record_error("s89_fork", hipGetLastError());
            if (forked) *forked = true;
            rc = gather_classes<0, XIN>(a, cs, nullptr);
        }
        if (!join) return rc;
        // joined even after a failed launch: later work on st must not overtake a side stream
        const int rj = join_side(st);
        return rc ? rc : rj;
    }

    // Makes st wait for everything enqueued so far on the device's side streams.
    static int join_side(hipStream_t st) {
        std::lock_guard<std::mutex> lock(g_fork_mu);
        ForkSet *fs = fork_set(st);
        if (!fs) return DSORT_OK;
        int rj = DSORT_OK;
        for (int i = 0; i < kForkStreams; ++i)
            if (hipEventRecord(fs->join[i], fs->side[i]) != hipSuccess ||
                hipStreamWaitEvent(st, fs->join[i], 0) != hipSuccess)
                rj = record_error("s89_join", hipGetLastError());
        return rj;
    }
    struct SideJoin {  // joins on scope exit when armed
        hipStream_t st;
        bool armed = false;
        ~SideJoin() {
            if (armed) (void)join_side(st);
        }
    };

    // Step 4 for one level.  G > 0 segments sorted one workgroup each, or (global) the single
    // segment's m*s samples by chunk sorts plus merge rounds ending in `sorted`.
    static int sort_samples(const SC *samp, SC *sorted, SC *tmp, SegView sv, uint32_t L,
                            uint32_t s, uint32_t G, uint32_t total, uint32_t *status,
                            hipStream_t st, bool global, uint32_t rounds, Timing *tm,
                            const char *name, const char *name_merge) {
        if (!global) {
            DS_LAUNCH(name, (k_sort_samples<SC, SE, SCAP>), dim3(G), dim3(SCAP / SE), samp,
                      sorted, sv, L, s, 0u, status);
            return DSORT_OK;
        }
        const uint32_t chunks = (total + SCAP - 1) / SCAP;
        SC *x = (rounds % 2 == 0) ? sorted : tmp;  // the last round must land in `sorted`
        SC *y = (rounds % 2 == 0) ? tmp : sorted;
        DS_LAUNCH(name, (k_sort_samples<SC, SE, SCAP>), dim3(chunks), dim3(SCAP / SE), samp, x,
                  sv, L, s, total, status);
        for (uint32_t run = SCAP; run < total; run <<= 1) {
            DS_LAUNCH(name_merge, (k_merge_round<SC, ME, MCAP>), dim3((total + MCAP - 1) / MCAP),
                      dim3(MCAP / ME),
                      (const SC *)x, y, total, run);
            SC *t = x;
            x = y;
            y = t;
        }
        return DSORT_OK;
    }

    // Segmented sort: every segment [off[g], off[g+1]) sorted on its own.  Segments that fit a
    // bucket workgroup are sorted in place as one-piece buckets; the others run one level of
    // Algorithm 1 together (the segmented kernels of the second level), sublists sorted into the
    // workspace copy and gathered back per bucket.
    static int run_segmented(const SegGeom &g, void *d_keys, uint32_t *d_vals,
                             const uint64_t *d_off, void *d_ws, hipStream_t st, Timing *tm,
                             uint32_t mask, bool fork) {
        char *ws = (char *)d_ws;
        uint32_t *status = (uint32_t *)(ws + g.o_status);
        DS_LAUNCH("init", k_init, dim3(1), dim3(64), status);
        K *keys = (K *)d_keys;
        const uint32_t n = (uint32_t)g.n;
        const uint32_t S = (uint32_t)g.S;
        uint4 *small_b = (uint4 *)(ws + g.o_small_b);
        uint32_t *spiece = (uint32_t *)(ws + g.o_spiece);
        uint32_t *slists = (uint32_t *)(ws + g.o_slists);
        // counters of the one-piece classes follow those of the final buckets
        const Classes scls = classes(status + kMaxClasses, slists, S);
        SegClassArgs ca{};
        ca.n = g.nclasses;
        for (uint32_t c = 0; c < g.nclasses; ++c) {
            const SegClassGeom &q = g.cls[c];
            ca.hi[c] = (uint32_t)q.hi;
            ca.L[c] = q.L;
            ca.gmax[c] = q.gmax;
            ca.tab[c] = (uint4 *)(ws + q.o_tab);
            ca.tile_off[c] = (uint32_t *)(ws + q.o_tileoff);
        }
        DS_LAUNCH("seg_prepare", k_seg_prepare, dim3(1), dim3(1024), d_off, S, n,
                  (uint32_t)g.max_seg, g.small_cap, ca, small_b, spiece, scls, status);
        // One-piece buckets in place (a workgroup reads its whole segment before writing).
        // When forked they keep running beside the long segments' Steps 1-7, which touch other
        // items and other counters; the first long class's own fork and join, or `side` on the
        // way out, joins them.
        SideJoin side{st};
        if (mask & kRunSmall) {
            GatherArgs a{keys, keys, d_vals, d_vals, small_b, spiece, spiece, scls.count, slists,
                         S, n, status};
            int rc0 = launch_classes<F32>(a, st, tm, fork, false, &side.armed);
            if (rc0) return rc0;
        }
        K *wkeys = (K *)(ws + g.o_wkeys);
        uint32_t *wvals = V ? (uint32_t *)(ws + g.o_wvals) : nullptr;
        SC *samp = (SC *)(ws + g.o_samp);
        SC *sorted = (SC *)(ws + g.o_samp_sorted);
        uint32_t *counts = (uint32_t *)(ws + g.o_counts);
        uint32_t *offs = (uint32_t *)(ws + g.o_offs);
        uint32_t *pdst = (uint32_t *)(ws + g.o_pdst);
        uint32_t *psrc = (uint32_t *)(ws + g.o_psrc);
        uint4 *finals = (uint4 *)(ws + g.o_final);
        uint32_t *lists = (uint32_t *)(ws + g.o_lists);
        bool first = true;
        for (uint32_t c = 0; c < g.nclasses; ++c) {
            const SegClassGeom &q = g.cls[c];
            if (!(mask & (1u << c)) || q.gmax == 0) continue;
            const Classes fcls = classes(status, lists, q.gmax * q.s);
            if (!first) DS_LAUNCH("seg_clear", k_clear_counters, dim3(1), dim3(64), fcls.count,
                                  (uint32_t)CC::n);
            first = false;
            const SegView sv{ca.tab[c], ca.tile_off[c], q.gmax, 0, n, q.tiles_max};
            {
                TileArgs a{keys, wkeys, d_vals, wvals, sv, q.L, q.s, samp, status};
                DS_LAUNCH("s123_local_sort", (k_tile<K, V, TE, TCAP, MODE_SAMPLE, F32, false>),
                          dim3(q.tiles_max), dim3(q.L / TE), a);
            }
            int rc = sort_samples(samp, sorted, nullptr, sv, q.L, q.s, q.gmax, 0, status, st,
                                  false, 0, tm, "s4_sample_sort", "s4_sample_merge");
            if (rc) return rc;
            DS_LAUNCH("s56_rank", (k_rank<K, V>), dim3(q.tiles_max), dim3(256),
                      (const K *)wkeys, (const void *)sorted, (const void *)samp, counts, sv,
                      q.L, q.s, 0u, (const K *)nullptr);
            DS_LAUNCH("s7_scan", k_scan_seg, dim3(q.gmax), dim3(256), (const uint32_t *)counts,
                      offs, pdst, psrc, sv, q.L, q.s, finals, fcls);
            GatherArgs a{wkeys, keys, wvals, d_vals, finals, pdst, psrc, fcls.count, lists,
                         q.gmax * q.s, n, status};
            rc = launch_classes(a, st, tm, fork);
            if (rc) return rc;
        }
        return DSORT_OK;
    }

    static int run(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws, hipStream_t st,
                   Timing *tm) {
        char *ws = (char *)d_ws;
        uint32_t *status = (uint32_t *)(ws + g.o_status);
        DS_LAUNCH("init", k_init, dim3(1), dim3(64), status);
        K *keys = (K *)d_keys;
        const uint32_t n = (uint32_t)g.n;
        if (g.levels == 0) {
            TileArgs a{keys, keys, d_vals, d_vals, SegView{nullptr, nullptr, 1, n, n, 0}, 0, 0,
                       nullptr, status};
            DS_LAUNCH("s9_bucket_sort", (k_tile<K, V, FE, FCAP, MODE_FINAL, F32, F32>), dim3(1),
                      dim3(FCAP / FE), a);
            return DSORT_OK;
        }
        K *wkeys = (K *)(ws + g.o_wkeys);
        uint32_t *wvals = V ? (uint32_t *)(ws + g.o_wvals) : nullptr;
        SC *samp = (SC *)(ws + g.o_samp);
        SC *sorted = (SC *)(ws + g.o_samp_sorted);
        SC *tmp = (SC *)(ws + g.o_samp_tmp);
        uint32_t *counts = (uint32_t *)(ws + g.o_counts);
        uint32_t *offs = (uint32_t *)(ws + g.o_offs);
        uint32_t *pdst = (uint32_t *)(ws + g.o_pdst);
        uint32_t *psrc = (uint32_t *)(ws + g.o_psrc);
        uint32_t *partial = (uint32_t *)(ws + g.o_partial);
        uint4 *buckets1 = (uint4 *)(ws + g.o_buckets1);
        uint32_t *tileoff2 = g.levels == 2 ? (uint32_t *)(ws + g.o_tileoff2) : nullptr;
        const SegView sv1{nullptr, nullptr, 1, n, n, g.m1};
        // One level: the sorted sublists go to the workspace copy, and the fused Steps 8-9
        // gather from there into keys.  Two levels: sorted in place, gathered piece by piece
        // into the second level's sorted sublists in the copy.
        K *tiles = g.levels == 1 ? wkeys : keys;
        uint32_t *tvals = g.levels == 1 ? wvals : d_vals;

        // Randomized samples (level 1 only): buckets beyond bucket_limit are listed here and
        // relocated as contiguous ranges for a further run (run_pipeline).
        const uint32_t rnd = g.random ? 1u : 0u;
        uint32_t *ovf_count = rnd ? status + kOverflowWord : nullptr;
        uint32_t *ovf_list = rnd ? (uint32_t *)(ws + g.o_ovf) : nullptr;
        const uint32_t limit = rnd ? g.bucket_limit : 0xFFFFFFFFu;

        // Steps 1-3
        {
            TileArgs a{keys, tiles, d_vals, tvals, sv1, g.L1, g.s1, samp, status, nullptr,
                       nullptr, g.seed, rnd, g.o_idx1 ? (void *)(ws + g.o_idx1) : nullptr};
            DS_LAUNCH("s123_local_sort", (k_tile<K, V, TE, TCAP, MODE_SAMPLE, F32, false>),
                      dim3(g.m1), dim3(g.L1 / TE), a);
        }
        // Step 4
        int rc = sort_samples(samp, sorted, tmp, sv1, g.L1, g.s1, 1, g.m1 * g.s1, status, st,
                              g.samp_global, g.samp_rounds, tm, "s4_sample_sort",
                              "s4_sample_merge");
        if (rc) return rc;
        // Steps 5-6
        DS_LAUNCH("s56_rank", (k_rank<K, V>), dim3(g.m1), dim3(256), (const K *)tiles,
                  (const void *)sorted, (const void *)samp, counts, sv1, g.L1, g.s1, rnd,
                  g.o_idx1 ? (const K *)(ws + g.o_idx1) : (const K *)nullptr);
        // Step 7
        DS_LAUNCH("s7_scan_colsum", k_scan_partial, dim3(g.scan_nrb), dim3(256),
                  (const uint32_t *)counts, partial, g.m1, g.s1, g.scan_rb);
        uint32_t *lists = (uint32_t *)(ws + g.o_lists);
        const Classes cls = classes(status, lists, g.final_buckets);
        Classes none{};
        DS_LAUNCH("s7_scan_mid", k_scan_mid, dim3(1), dim3(1024), partial, g.scan_nrb, g.m1,
                  g.s1, n, buckets1, tileoff2, g.L2, g.levels == 1 ? cls : none, limit,
                  ovf_count, ovf_list);
        DS_LAUNCH("s7_scan_update", k_scan_apply, dim3(g.scan_nrb), dim3(256),
                  (const uint32_t *)counts, (const uint32_t *)partial, (const uint4 *)buckets1,
                  offs, pdst, psrc, g.m1, g.s1, g.scan_rb, g.L1);
        if (rnd) {
            // one level: the listed buckets go straight to their places in keys; two levels:
            // to the workspace copy, which the second level fills only at the other buckets
            DS_LAUNCH("s8_reloc_listed", (k_reloc_listed<K>), dim3(kListedGrid), dim3(256),
                      (const K *)tiles, g.levels == 1 ? keys : wkeys, tvals,
                      V ? (g.levels == 1 ? d_vals : wvals) : nullptr, (const uint4 *)buckets1,
                      (const uint32_t *)pdst, (const uint32_t *)psrc,
                      (const uint32_t *)ovf_count, (const uint32_t *)ovf_list, g.s1, g.m1, n,
                      (g.levels == 1 && F32) ? 1u : 0u);
        }

        if (g.levels == 1) {
            // Steps 8-9 fused: gather every bucket's pieces, merge them, write into keys.
            GatherArgs a{wkeys, keys, wvals, d_vals, buckets1, pdst, psrc, status + 1, lists,
                         g.final_buckets, n, status};
            return launch_classes(a, st, tm, false);
        }

        // Step 9 as a second level: Algorithm 1 on every bucket of level 1, its sublists
        // gathered from the level-1 pieces (Step 8 fused into Step 1) and written sorted into
        // the workspace copy; its own fused Steps 8-9 write the final order into keys.
        const SegView sv2{buckets1, tileoff2, g.s1, 0, n, g.tiles2max};
        SC *samp2 = (SC *)(ws + g.o_samp2);
        SC *sorted2 = (SC *)(ws + g.o_samp2_sorted);
        uint32_t *counts2 = (uint32_t *)(ws + g.o_counts2);
        uint32_t *offs2 = (uint32_t *)(ws + g.o_offs2);
        uint32_t *pdst2 = (uint32_t *)(ws + g.o_pdst2);
        uint32_t *psrc2 = (uint32_t *)(ws + g.o_psrc2);
        uint4 *finals = (uint4 *)(ws + g.o_final);
        {
            TileArgs a{keys, wkeys, d_vals, wvals, sv2, g.L2, g.s2, samp2, status, pdst, psrc, 0, 0,
                       g.o_idx2 ? (void *)(ws + g.o_idx2) : nullptr};
            DS_LAUNCH("s8_l2_s123_gather_sort",
                      (k_tile<K, V, TE, TCAP, MODE_SAMPLE, false, false, true>),
                      dim3(g.tiles2max), dim3(g.L2 / TE), a);
        }
        rc = sort_samples(samp2, sorted2, nullptr, sv2, g.L2, g.s2, g.s1, 0, status, st, false, 0,
                          tm, "l2_s4_sample_sort", "l2_s4_sample_merge");
        if (rc) return rc;
        DS_LAUNCH("l2_s56_rank", (k_rank<K, V>), dim3(g.tiles2max), dim3(256), (const K *)wkeys,
                  (const void *)sorted2, (const void *)samp2, counts2, sv2, g.L2, g.s2, 0u,
                  g.o_idx2 ? (const K *)(ws + g.o_idx2) : (const K *)nullptr);
        DS_LAUNCH("l2_s7_scan", k_scan_seg, dim3(g.s1), dim3(256), (const uint32_t *)counts2,
                  offs2, pdst2, psrc2, sv2, g.L2, g.s2, finals, cls);
        GatherArgs a{wkeys, keys, wvals, d_vals, finals, pdst2, psrc2, status + 1, lists,
                     g.final_buckets, n, status};
        rc = launch_classes(a, st, tm, false);
        if (rc || !rnd) return rc;
        DS_LAUNCH("s8_copy_listed", (k_copy_listed<K>), dim3(kListedGrid), dim3(256),
                  (const K *)wkeys, keys, (const uint32_t *)wvals, V ? d_vals : nullptr,
                  (const uint4 *)buckets1, (const uint32_t *)ovf_count,
                  (const uint32_t *)ovf_list, g.s1, n, F32 ? 1u : 0u);
        return DSORT_OK;
    }
};

}  // namespace

void timing_reset(Timing &t) {
    t.used = 0;
    t.recs.clear();
}

void timing_destroy(Timing &t) {
    for (void *e : t.pool) hipEventDestroy((hipEvent_t)e);
    t.pool.clear();
    t.recs.clear();
    t.used = 0;
}

int timing_summary(Timing &t, const char **names, float *avg_ms, uint32_t *launches,
                   int capacity, int *count) {
    std::vector<const char *> nm;
    std::vector<double> sum;
    std::vector<uint32_t> cnt;
    for (const StageRec &r : t.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, (hipEvent_t)r.ev0, (hipEvent_t)r.ev1) != hipSuccess)
            return DSORT_E_HIP;
        size_t k = 0;
        while (k < nm.size() && nm[k] != r.name) ++k;
        if (k == nm.size()) {
            nm.push_back(r.name);
            sum.push_back(0.0);
            cnt.push_back(0);
        }
        sum[k] += ms;
        cnt[k] += 1;
    }
    const int c = (int)nm.size();
    for (int k = 0; k < c && k < capacity; ++k) {
        if (names) names[k] = nm[k];
        if (avg_ms) avg_ms[k] = (float)(sum[k] / cnt[k]);
        if (launches) launches[k] = cnt[k];
    }
    *count = c;
    return DSORT_OK;
}

// Batch staging for the served stream: copies request g's items between its own buffers
// (keys at src_keys[g], values at src_vals[g]) and positions [off[g], off[g+1]) of one staging
// array, in either direction.  Each workgroup moves one chunk of kPackChunk staging positions,
// finding the request of its first position by bisection and walking forward from there.
constexpr uint32_t kPackChunk = 8192;

template <class K>
__global__ __launch_bounds__(256) void k_pack(const uint64_t *src_keys, const uint64_t *src_vals,
                                              const uint64_t *off, uint32_t S, K *stage_keys,
                                              uint32_t *stage_vals, uint32_t unpack) {
    const uint64_t total = off[S];
    const uint64_t c0 = (uint64_t)blockIdx.x * kPackChunk;
    if (c0 >= total) return;
    const uint64_t c1 = min(total, c0 + kPackChunk);
    uint32_t lo = 0, hi = S - 1;  // last g with off[g] <= c0
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= c0) lo = mid; else hi = mid - 1;
    }
    for (uint32_t g = lo; g < S && off[g] < c1; ++g) {
        const uint64_t a = max(off[g], c0), b = min(off[g + 1], c1);
        K *uk = (K *)src_keys[g];
        uint32_t *uv = (uint32_t *)src_vals[g];
        for (uint64_t x = a + threadIdx.x; x < b; x += blockDim.x) {
            const uint64_t r = x - off[g];
            if (unpack) {
                uk[r] = stage_keys[x];
                if (stage_vals) uv[r] = stage_vals[x];
            } else {
                stage_keys[x] = uk[r];
                if (stage_vals) stage_vals[x] = uv[r];
            }
        }
    }
}

int launch_pack(int key_bytes, const uint64_t *d_src_keys, const uint64_t *d_src_vals,
                const uint64_t *d_off, uint32_t S, uint64_t total, void *stage_keys,
                uint32_t *stage_vals, bool unpack, void *stream) {
    if (S == 0 || total == 0) return DSORT_OK;
    const uint64_t chunks = (total + kPackChunk - 1) / kPackChunk;
    if (chunks > 0x7FFFFFFFu) return DSORT_E_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    if (key_bytes == 8)
        hipLaunchKernelGGL((k_pack<uint64_t>), dim3((uint32_t)chunks), dim3(256), 0, st,
                           d_src_keys, d_src_vals, d_off, S, (uint64_t *)stage_keys, stage_vals,
                           unpack ? 1u : 0u);
    else
        hipLaunchKernelGGL((k_pack<uint32_t>), dim3((uint32_t)chunks), dim3(256), 0, st,
                           d_src_keys, d_src_vals, d_off, S, (uint32_t *)stage_keys, stage_vals,
                           unpack ? 1u : 0u);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_error(unpack ? "unpack" : "pack", hipGetErrorName(e), hipGetErrorString(e));
        return DSORT_E_HIP;
    }
    return DSORT_OK;
}

int run_segmented(const SegGeom &g, void *d_keys, uint32_t *d_vals, const uint64_t *d_off,
                  void *d_ws, void *stream, Timing *tm, uint32_t mask, bool fork) {
    hipStream_t st = (hipStream_t)stream;
    if (g.S == 0 || g.n == 0) return DSORT_OK;
    (void)hipGetLastError();
    if (tm && !tm->enabled) tm = nullptr;
    switch (g.key_type) {
        case DSORT_U32:
            return g.values ? Pipeline<uint32_t, true, false>::run_segmented(g, d_keys, d_vals,
                                                                            d_off, d_ws, st, tm, mask, fork)
                            : Pipeline<uint32_t, false, false>::run_segmented(g, d_keys, d_vals,
                                                                             d_off, d_ws, st, tm, mask, fork);
        case DSORT_F32:
            return g.values ? Pipeline<uint32_t, true, true>::run_segmented(g, d_keys, d_vals,
                                                                           d_off, d_ws, st, tm, mask, fork)
                            : Pipeline<uint32_t, false, true>::run_segmented(g, d_keys, d_vals,
                                                                            d_off, d_ws, st, tm, mask, fork);
        case DSORT_U64:
            return g.values ? Pipeline<uint64_t, true, false>::run_segmented(g, d_keys, d_vals,
                                                                            d_off, d_ws, st, tm, mask, fork)
                            : Pipeline<uint64_t, false, false>::run_segmented(g, d_keys, d_vals,
                                                                             d_off, d_ws, st, tm, mask, fork);
        default:
            return DSORT_E_INVALID;
    }
}

static int run_geom(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws, hipStream_t st,
                    Timing *tm) {
    switch (g.key_type) {
        case DSORT_U32:
            return g.values ? Pipeline<uint32_t, true, false>::run(g, d_keys, d_vals, d_ws, st, tm)
                            : Pipeline<uint32_t, false, false>::run(g, d_keys, d_vals, d_ws, st, tm);
        case DSORT_F32:
            return g.values ? Pipeline<uint32_t, true, true>::run(g, d_keys, d_vals, d_ws, st, tm)
                            : Pipeline<uint32_t, false, true>::run(g, d_keys, d_vals, d_ws, st, tm);
        case DSORT_U64:
            return g.values ? Pipeline<uint64_t, true, false>::run(g, d_keys, d_vals, d_ws, st, tm)
                            : Pipeline<uint64_t, false, false>::run(g, d_keys, d_vals, d_ws, st, tm);
        default:
            return DSORT_E_INVALID;
    }
}

__global__ void k_set_word(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// The further run of a randomized call: reads back the level-1 buckets that the pipeline routed
// past its normal path (already relocated, unsorted, to their final ranges in the keys) and
// sorts each range in place with the deterministic automatic plan, in the same workspace (the
// caller sized it for that).  Waits for the stream once, plus once more when buckets were
// routed.  A call whose kernels raised status flags is left as it is (the flags stay for the
// caller); after further runs the status page holds their flags and the routed-bucket count.
static int finish_random(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws,
                         hipStream_t st, Timing *tm) {
    const char *ws = (const char *)d_ws;
    uint32_t page[64];
    if (hipMemcpyAsync(page, ws + g.o_status, sizeof(page), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return record_error("random_readback", hipGetLastError());
    const uint32_t cnt = page[kOverflowWord];
    if (cnt == 0 || page[0] != 0) return DSORT_OK;
    if (cnt > g.s1) return record_error("random_readback", hipErrorInvalidValue);
    std::vector<uint32_t> list(cnt);
    std::vector<uint4> table(g.s1);
    if (hipMemcpyAsync(list.data(), ws + g.o_ovf, 4ull * cnt, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(table.data(), ws + g.o_buckets1, sizeof(uint4) * g.s1,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return record_error("random_readback", hipGetLastError());
    const size_t kb = g.caps.key_bytes;
    for (uint32_t b : list) {
        if (b >= g.s1) return record_error("random_readback", hipErrorInvalidValue);
        const uint4 d = table[b];
        if ((uint64_t)d.x + d.y > g.n) return record_error("random_readback", hipErrorInvalidValue);
        Geom h;
        const dsort_tuning_t automatic{};
        int rc = make_geom(g.key_type, g.values, d.y, automatic, h);
        if (rc != DSORT_OK) return rc;
        if (h.levels < 0) continue;
        rc = run_geom(h, (char *)d_keys + kb * d.x, d_vals ? d_vals + d.x : nullptr, d_ws, st, tm);
        if (rc != DSORT_OK) return rc;
    }
    hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, st,
                       (uint32_t *)((char *)d_ws + g.o_status) + kOverflowWord, cnt);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DSORT_OK : record_error("random_count", e);
}

int run_pipeline(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws, void *stream,
                 Timing *tm) {
    hipStream_t st = (hipStream_t)stream;
    if (g.levels < 0) return DSORT_OK;
    (void)hipGetLastError();  // do not attribute an earlier caller's error to this call
    if (g.n > 0xFFFFFFFFull) return DSORT_E_INVALID;
    if (tm && !tm->enabled) tm = nullptr;
    if (g.random) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            return DSORT_E_UNSUPPORTED;  // the further run needs a read-back
        }
    }
    const int rc = run_geom(g, d_keys, d_vals, d_ws, st, tm);
    if (rc != DSORT_OK || !g.random) return rc;
    return finish_random(g, d_keys, d_vals, d_ws, st, tm);
}

}  // namespace dsort
