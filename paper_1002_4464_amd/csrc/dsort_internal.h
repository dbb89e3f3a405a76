// Internal declarations shared by the host planner (plan.cpp) and the HIP pipeline
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dsort.h"

namespace dsort {

// Per (key type, values) capacities of the workgroup sorts.  They must match the kernel
// instantiations in kernels.hip.
struct Caps {
    uint32_t tile_max;   // largest sublist length L one workgroup sorts in Step 2
    uint32_t tile_e;     // items per thread of that sort
    uint32_t final_cap;  // largest bucket one workgroup sorts in Step 9
    uint32_t final_e;
    uint32_t samp_cap;   // largest sample set one workgroup sorts in Step 4
    uint32_t samp_e;
    uint32_t key_bytes;
    uint32_t samp_bytes; // bytes of one sample composite
};

Caps caps_for(int key_type, bool values);

// Everything one call needs: the level structure, the launch geometry and the workspace map.
struct Geom {
    int key_type = 0;
    bool values = false;
    uint64_t n = 0;
    int levels = -1;  // -1: nothing to do (n <= 1); 0: one tile; 1; 2
    Caps caps{};

    // level 1
    uint32_t L1 = 0, s1 = 0, m1 = 0;
    uint32_t beta1 = 0;
    bool samp_global = false;  // Step 4 as chunk sorts + merge rounds
    uint32_t samp_rounds = 0;
    bool scan_large = false;   // Step 7 as three kernels over row blocks
    uint32_t scan_rb = 0, scan_nrb = 0;
    // level 2
    uint32_t L2 = 0, s2 = 0, m2max = 0, tiles2max = 0;
    uint32_t final_buckets = 0;
    uint32_t plan_rule = 0;  // which rule chose (s1, s2): 0 preferred, 1 smallest feasible
    // randomized samples at level 1 (the comparison method): no bucket bound, so level-1
    // buckets of more than bucket_limit real items skip Step 9's normal path and are sorted by
    // a further deterministic run afterwards
    bool random = false;
    uint64_t seed = 0;
    uint32_t bucket_limit = 0;

    // workspace byte offsets
    size_t o_status = 0, o_wkeys = 0, o_wvals = 0;
    size_t o_samp = 0, o_samp_sorted = 0, o_samp_tmp = 0;
    size_t o_counts = 0, o_offs = 0, o_pdst = 0, o_psrc = 0, o_partial = 0;
    size_t o_buckets1 = 0, o_tileoff2 = 0;
    size_t o_samp2 = 0, o_samp2_sorted = 0, o_counts2 = 0, o_offs2 = 0, o_pdst2 = 0, o_psrc2 = 0;
    size_t o_final = 0, o_lists = 0;
    size_t o_ovf = 0;  // randomized: the level-1 buckets routed to the further run
    // rank index of each level's sorted sublists: the key at every 16th rank (0 = none)
    size_t o_idx1 = 0, o_idx2 = 0;
    size_t total = 0;
};

// Word of the workspace's status page that counts the level-1 buckets of a randomized call
// routed to the further run (cleared by the pipeline's first kernel).
constexpr uint32_t kOverflowWord = 40;

// Segmented sorts: segments of at most small_cap items are sorted as one-piece buckets; the
// longer ones are split by length into classes (lengths in (lo, hi]), each running one level of
// Algorithm 1 with its own sublist length L and samples per sublist s.
constexpr int kMaxSegClasses = 4;

// Tuning of the long-segment classes.  classes = 0: one class with the defaults.  Class c holds
// lengths in (upper[c-1], upper[c]] (upper[-1] = small_cap); the last class also takes every
// longer segment.  L[c] = 0: the largest tile; s[c] = 0: the smallest s that bounds the buckets.
struct SegTuning {
    uint32_t classes = 0;
    uint64_t upper[kMaxSegClasses] = {};
    uint32_t L[kMaxSegClasses] = {};
    uint32_t s[kMaxSegClasses] = {};
};

struct SegClassGeom {
    uint64_t lo = 0, hi = 0;  // lengths in (lo, hi]
    uint32_t L = 0, s = 0, gmax = 0, tiles_max = 0;
    uint64_t beta = 0;        // bucket bound of a segment of hi items
    size_t o_tab = 0, o_tileoff = 0;
};

struct SegGeom {
    int key_type = 0;
    bool values = false;
    uint64_t n = 0, S = 0, max_seg = 0;
    Caps caps{};
    uint32_t small_cap = 0;
    uint32_t nclasses = 0;  // classes with room for at least one segment
    SegClassGeom cls[kMaxSegClasses];
    size_t o_status = 0, o_small_b = 0, o_spiece = 0, o_slists = 0;
    // shared by the classes (they run one after the other)
    size_t o_wkeys = 0, o_wvals = 0, o_samp = 0, o_samp_sorted = 0, o_counts = 0, o_offs = 0;
    size_t o_pdst = 0, o_psrc = 0, o_final = 0, o_lists = 0;
    size_t total = 0;
};

// Most segments one segmented call accepts (the set-up walks them in one workgroup).
constexpr uint64_t kMaxSegments = 1u << 24;

// Longest segment the one-level segmented plan accepts for this key layout.
uint64_t seg_limit(int key_type, bool values);


// Computes the geometry for n items.  Returns DSORT_OK or DSORT_E_UNSUPPORTED.
int make_geom(int key_type, bool values, uint64_t n, const dsort_tuning_t &tuning, Geom &g);

// Optional per-kernel timing: every launch of a sorting call is bracketed by two HIP events
// (hipEvent_t stored as void*) recorded on the call's stream.
struct StageRec {
    const char *name;
    void *ev0;
    void *ev1;
};
struct Timing {
    bool enabled = false;
    std::vector<void *> pool;  // events, reused across resets
    size_t used = 0;
    std::vector<StageRec> recs;
};
void timing_reset(Timing &t);
void timing_destroy(Timing &t);
// Averages the recorded launches per stage name (in first-seen order).  Needs the stream of
// the recorded calls to have been synchronised.  Returns DSORT_OK or DSORT_E_HIP.
int timing_summary(Timing &t, const char **names, float *avg_ms, uint32_t *launches,
                   int capacity, int *count);

// Enqueues the whole pipeline (kernels.hip).  Pointers are device pointers; tm may be null.
int make_seg_geom(int key_type, bool values, uint64_t n, uint64_t S, uint64_t max_seg,
                  const SegTuning &tu, SegGeom &g);
// Smallest s for m sublists of L items (0 if none): buckets within one workgroup, samples
// within the one-workgroup sample sort.
uint64_t seg_samples(const Caps &c, uint64_t m, uint64_t L);
// Workspace enough for every tuning the autotuner may pick (and the default one).
size_t seg_workspace_bound(int key_type, bool values, uint64_t n, uint64_t S, uint64_t max_seg);
// The class split the autotuner uses: lengths in (small_cap, 4 small_cap], (4, 16 small_cap], ...
SegTuning seg_default_split(int key_type, bool values, uint64_t max_seg);
// Candidate sublist lengths of the autotuner, largest first (count returned).
int seg_candidate_L(const Caps &c, uint32_t *out);
constexpr uint32_t kRunSmall = 1u << 31;  // run_segmented mask bit of the one-piece segments
// fork: run the bucket size classes on side streams as well (joined before return); off for
// callers that already run several sorts side by side.
int run_segmented(const SegGeom &g, void *d_keys, uint32_t *d_vals, const uint64_t *d_off,
                  void *d_ws, void *stream, Timing *tm, uint32_t mask = 0xFFFFFFFFu,
                  bool fork = false);
// Copies between requests' own buffers and a staging array (served-stream batches).
int launch_pack(int key_bytes, const uint64_t *d_src_keys, const uint64_t *d_src_vals,
                const uint64_t *d_off, uint32_t S, uint64_t total, void *stage_keys,
                uint32_t *stage_vals, bool unpack, void *stream);
int run_pipeline(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws, void *stream,
                 Timing *tm);

// Last failure of this thread, for dsort_last_error() (plan.cpp).
void set_last_error(const char *stage, const char *name, const char *text);

constexpr uint64_t kMaxItems = (1ull << 32) - (1ull << 16);

int plan_set_seg_tuning(dsort_plan_s *plan, const SegTuning &tu);

// Persisted autotuner results (tune_cache.cpp): one tuning per (device, key type, values,
// segment class = ceil(log2(max_segment))) in a text file.
struct TuneKey {
    std::string device;  // architecture, marketing name and CU count
    int key_type = 0;
    bool values = false;
    uint32_t seg_class = 0;
};
uint32_t tune_seg_class(uint64_t max_segment);
bool tune_cache_lookup(const char *path, const TuneKey &key, SegTuning &out);
bool tune_cache_store(const char *path, const TuneKey &key, const SegTuning &t);

}  // namespace dsort

// Host state of a plan (dsort_plan_t).
struct dsort_plan_s {
    uint32_t magic;
    int key_type;
    int values;
    uint64_t max_items;
    uint64_t max_segments;
    dsort_tuning_t tuning;
    size_t workspace;
    dsort::Geom last;  // geometry cache of the last n
    dsort::Timing timing;
    dsort::SegTuning seg_tuning;  // long-segment classes of dsort_segmented
};

namespace dsort {
constexpr uint32_t kPlanMagic = 0x44534f52u;  // "DSOR"
inline bool plan_valid(const dsort_plan_s *p) { return p && p->magic == kPlanMagic; }
}  // namespace dsort
