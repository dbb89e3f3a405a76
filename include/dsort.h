/*
 * dsort: deterministic sample sort ("GPU Bucket Sort", Algorithm 1 of Dehne & Zaboli,
 * "Deterministic Sample Sort For GPUs", Section 4) for AMD Instinct MI355X (gfx950).
 *
 * Plain C ABI: every entry point is extern "C", takes plain pointers and sizes, and never
 * throws.  Device pointers are HIP device allocations owned by the caller; `stream` is a
 * hipStream_t passed as void* (NULL = the default stream).  Sorting calls only enqueue work on
 * `stream` and return; kernel faults surface at the caller's next synchronisation.
 *
 * Problem statement (Algorithm 1, "Input"/"Output"): an array A of n items in device memory is
 * sorted in place.  Key order: uint32 and uint64 keys by unsigned value; float32 keys by IEEE
 * 754 totalOrder of their bit patterns (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN; the
 * output holds the input bit patterns, permuted).  Key/value sorts are stable: equal keys keep
 * their input order.  Algorithm 1 compares items under the total order (key, sublist, rank), so
 * the bucket-size bound of Section 4 holds for any input, repeated keys included.
 *
 * Status codes are the DSORT_* values below; dsort_strerror() describes them.
 */
#ifndef DSORT_H
#define DSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types. */
enum {
    DSORT_U32 = 1, /* uint32_t keys */
    DSORT_U64 = 2, /* uint64_t keys */
    DSORT_F32 = 3  /* float keys, ordered by IEEE totalOrder */
};

/* Status codes (0 = success, negative = failure). */
enum {
    DSORT_OK = 0,
    DSORT_E_INVALID = -1,     /* bad argument: NULL pointer, unknown type, n > plan maximum, ... */
    DSORT_E_UNSUPPORTED = -2, /* valid request the library cannot serve (e.g. tuning infeasible) */
    DSORT_E_NOMEM = -3,       /* host allocation failed */
    DSORT_E_HIP = -4,         /* a HIP runtime call or kernel launch failed */
    DSORT_E_CAPACITY = -5,    /* request larger than a configured capacity */
    DSORT_E_TICKET = -6       /* unknown ticket */
};

/* Optional tuning.  Zero in a field means "choose automatically".
 *  sublist_len  L  of the first level (Step 1: the sublist length n/m): a power of two, or
 *                  a multiple of 1024 (512 for 64-bit keys with values), at most 16384 (8192
 *                  for 64-bit keys with values);
 *  samples      s  of the first level (Step 3: samples per sublist = number of buckets),
 *                  at most 1024, dividing L;
 *  sublist_len2, samples2: the same for the second level (Step 9 run as a segmented sort);
 *  levels       0 = auto, 1 = force one level (Step 9 sorts each bucket in one workgroup),
 *               2 = force two levels;
 *  sampling     0 = Algorithm 1 (Step 3 takes the last item of each of the s chunks of a
 *               sorted sublist, which bounds every bucket, Section 4); 1 = the randomized-
 *               splitter comparison method of Sections 1 and 3: Step 3 of the first level
 *               takes the items at s random sorted positions instead (sample k of sublist i at
 *               ((d >> 32) * L) >> 32, d = draw i*s + k of the SplitMix64 stream of `seed`,
 *               positions may repeat) and the last bucket is closed by +infinity.  Nothing
 *               then bounds a bucket: a first-level bucket larger than what its second step can
 *               take (one workgroup, or the second level's sublist count) is moved to its place
 *               as a contiguous range (Step 8) and sorted afterwards by a further run of
 *               Algorithm 1 (deterministic samples) on that range.  Finding such buckets costs
 *               one device-to-host read per call, so a randomized call waits for its own
 *               kernels (it synchronises `stream`) and cannot be captured into a graph.  The
 *               result is the same unique sorted order.  Plain sorts only (dsort_keys,
 *               dsort_pairs);
 *  seed         the randomized variant's stream seed. */
typedef struct {
    uint32_t sublist_len;
    uint32_t samples;
    uint32_t sublist_len2;
    uint32_t samples2;
    uint32_t levels;
    uint32_t sampling;
    uint64_t seed;
} dsort_tuning_t;

typedef struct dsort_plan_s *dsort_plan_t;

/* Plan a sort of up to `max_items` items of key type `key_type` (DSORT_U32/U64/F32), with
 * (`with_values` = 1) or without (0) a uint32 value per key.  `max_segments` bounds the
 * segment count of dsort_segmented (0 if unused, at most 2^24).  `tuning` may be NULL.
 * On success *out receives the plan (host memory, owned by the caller until
 * dsort_plan_destroy) and *workspace_bytes the size of the device workspace every call
 * with this plan needs.  The plan holds host state only and allocates no device memory.
 * Errors: DSORT_E_INVALID (NULL out/workspace_bytes, bad type, max_items above 2^32 - 2^16),
 * DSORT_E_UNSUPPORTED (the tuning cannot be realised, or max_items is beyond what two levels
 * of Algorithm 1 reach: 1,108,377,600 items for 32-bit keys, 554,188,800 for 32-bit keys with
 * values and for 64-bit keys, 286,326,784 for 64-bit keys with values), DSORT_E_NOMEM. */
int dsort_plan(dsort_plan_t *out, int key_type, int with_values, uint64_t max_items,
               uint64_t max_segments, const dsort_tuning_t *tuning, size_t *workspace_bytes);

/* Sort `n` keys at `d_keys` in place (Algorithm 1, Steps 1-9).  `d_workspace` must hold the
 * plan's workspace_bytes of device memory, 256-byte aligned; its contents on entry do not
 * matter and on return hold the intermediates of the last call (see dsort_plan_geometry).
 * n = 0 and n = 1 are no-ops.  Requires a plan made with with_values = 0.
 * Errors: DSORT_E_INVALID (NULL plan/pointers, n > max_items, plan with values),
 * DSORT_E_HIP (a launch failed).  One plan + workspace pair serves one stream at a time. */
int dsort_keys(dsort_plan_t plan, void *d_keys, uint64_t n, void *d_workspace, void *stream);

/* Stable sort of `n` (key, value) pairs in place: d_keys as for dsort_keys, d_values holds n
 * uint32 values that move with their keys; equal keys keep input order.  Requires a plan made
 * with with_values = 1.  Errors as for dsort_keys. */
int dsort_pairs(dsort_plan_t plan, void *d_keys, uint32_t *d_values, uint64_t n,
                void *d_workspace, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same sort as dsort_keys (with_values = 0) or
 * dsort_pairs (with_values = 1) under the automatic plan, with no plan and no caller workspace.
 * The workspace is a fixed device array of DSORT_NOALLOC_SCRATCH_BYTES inside the library, one
 * per GPU, created when the library's code is loaded on that GPU and held until the process
 * ends; the call itself allocates nothing, host or device.  `n` is limited to sizes whose
 * workspace (dsort_plan_geometry's workspace_bytes under the automatic plan) fits the array:
 * 13,801,792 uint32/float32 keys, 7,615,552 32-bit keys with values, 7,086,432 uint64 keys
 * and 4,755,104 uint64 keys with values.  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (two streams, two host threads) race and corrupt each other; calls
 * must be ordered (one stream, or synchronised).  The array keeps the last call's
 * intermediates; each call clears what it needs cleared on the device.
 * Errors: DSORT_E_INVALID (bad type, pointers, alignment, or d_values given for with_values =
 * 0), DSORT_E_CAPACITY (n above the limit; nothing is enqueued), DSORT_E_HIP. n <= 1: no-op. */
#define DSORT_NOALLOC_SCRATCH_BYTES (64u << 20)
int dsort_sort_noalloc(int key_type, int with_values, void *d_keys, uint32_t *d_values,
                       uint64_t n, void *stream);

/* Release a plan (NULL is accepted). */
int dsort_plan_destroy(dsort_plan_t plan);

/* Static description of the string for a status code (never NULL). */
const char *dsort_strerror(int status);

/* Details of the last DSORT_E_HIP failure on the calling thread: the pipeline stage whose launch
 * failed and the HIP error name and text ("" if none).  Valid until the thread's next failing
 * call. */
const char *dsort_last_error(void);

/* Geometry the plan uses for a call with `n` items, and where the intermediates of the first
 * level live inside the workspace after such a call (byte offsets from d_workspace).
 * levels: 0 = the whole input fits one workgroup tile and is sorted directly;
 *         1 = Algorithm 1 once, Step 9 sorts every bucket inside one workgroup;
 *         2 = Step 9 of the first level is itself Algorithm 1, run on every bucket.
 * Sample arrays hold composites (key, i*L + r) (32-bit keys: one uint64 (key << 32) | pos;
 * 64-bit keys: 16 bytes {uint64 key, uint32 pos, uint32 unused}).  Count and offset matrices
 * are m x s row-major uint32; row i belongs to sublist i; offsets are absolute positions. */
typedef struct {
    uint64_t n;
    uint32_t levels;
    uint32_t sublist_len, samples, sublists;       /* L, s, m of level 1 */
    uint32_t sublist_len2, samples2, max_tiles2;   /* L, s and a bound on sublists of level 2 */
    uint32_t bucket_capacity;                      /* largest bucket one workgroup sorts */
    uint32_t bucket_bound;                         /* 2 n'/s - m of level 1 */
    uint32_t sample_bytes;                         /* bytes per sample composite */
    uint32_t sample_sort_global;                   /* 1: Step 4 uses the multi-kernel merge */
    uint64_t off_status;          /* uint32 error flags raised by kernels (0 = none) */
    uint64_t off_samples;         /* level-1 samples in sublist order (Step 3) */
    uint64_t off_sorted_samples;  /* level-1 samples after Step 4 */
    uint64_t off_counts;          /* a_ij (Step 6) */
    uint64_t off_offsets;         /* l_ij (Step 7) */
    uint64_t off_buckets;         /* level-1 buckets as uint32 {begin, size, first piece, pieces} */
    uint64_t workspace_bytes;     /* bytes this n needs (<= the plan's workspace size) */
    /* Randomized sampling (tuning.sampling = 1) only, else 0: first-level buckets with more
     * than bucket_limit items skip the second step and are sorted by a further run; their
     * count (uint32) and their bucket indices (uint32 each) after a call. */
    uint32_t sampling;
    uint32_t bucket_limit;
    uint64_t off_overflow_count;
    uint64_t off_overflow_list;
} dsort_geometry_t;

int dsort_plan_geometry(dsort_plan_t plan, uint64_t n, dsort_geometry_t *out);

/* Segmented sort: sorts each of `num_segments` segments of the n-item arrays on its own, in
 * place, as if dsort_keys / dsort_pairs ran on each (same key order, same stability); one
 * call sorts them all, so many small sorts share the device.  Segment g is the item range
 * [d_offsets[g], d_offsets[g+1]) (CSR form: d_offsets is device memory holding num_segments + 1
 * non-decreasing uint64 values, all <= n, read on the device).  Items outside every segment
 * are left untouched.  d_values is NULL for keys-only plans and n uint32 values otherwise.
 * `max_segment` is a bound on every segment's length (0 = the limit below, or n if smaller);
 * it fixes the plan used for the long segments, so a tight bound saves work.
 *
 * Method (Algorithm 1 applied per segment, as in a second level of Step 9): a segment of at
 * most `small_capacity` items is one bucket, sorted inside one workgroup; every longer segment
 * runs one level of Algorithm 1 (sublists of L items, s samples per sublist, its own splitters
 * and buckets), all segments together in the same kernel launches.  A segment may hold at most
 * `segment_limit` items (dsort_segmented_geometry); longer ones need dsort_keys/dsort_pairs.
 *
 * The plan must have been made with max_segments >= num_segments and max_items >= n; the
 * workspace is the plan's.  Bad offsets are caught on the device and reported in the uint32
 * status word at workspace offset `off_status` (0 = clean run): offsets that decrease or
 * exceed n set the flag 0x10 and then no segment is sorted; a segment longer than max_segment
 * sets the flag 0x20 and is left as it is (the others are sorted).
 *
 * Streams: the call is ordered on `stream` like any other work on it.  Internally its bucket
 * sorts may also run on side streams (three per device, created by the library on the first
 * call made outside stream capture and kept for the process); the call ends by enqueueing on
 * `stream` a wait for them, so work enqueued on `stream` afterwards sees the sorted result.
 * A call made while `stream` is being captured into a graph runs everything on `stream` (the
 * side streams never enter a capture).  Calls from several host threads are safe; their
 * bucket sorts then share the side streams.
 * Errors: DSORT_E_INVALID (bad plan or pointer, misalignment, values given to a keys-only plan
 * or missing for a pairs plan, n or num_segments above the plan's), DSORT_E_UNSUPPORTED
 * (max_segment above segment_limit, or a plan with randomized sampling), DSORT_E_HIP.  n = 0 or num_segments = 0 is a no-op. */
int dsort_segmented(dsort_plan_t plan, void *d_keys, uint32_t *d_values, uint64_t n,
                    const uint64_t *d_offsets, uint64_t num_segments, uint64_t max_segment,
                    void *d_workspace, void *stream);

/* Geometry of a segmented call with these sizes (see dsort_segmented), under the plan's
 * current tuning.  Long segments (longer than small_capacity) are split by length into up to
 * four classes; class c holds lengths in (class_upper[c-1], class_upper[c]] (class_upper[-1] =
 * small_capacity) and runs one level of Algorithm 1 with its own L and s. */
typedef struct {
    uint64_t n, num_segments;
    uint64_t max_segment;           /* the bound used (after defaulting and clamping to n) */
    uint64_t segment_limit;         /* longest segment this key layout accepts */
    uint32_t small_capacity;        /* segments up to this size are sorted in one workgroup */
    uint32_t classes;               /* long-segment classes with room for a segment */
    uint64_t class_upper[4];
    uint32_t sublist_len[4];        /* L of each class */
    uint32_t samples[4];            /* s of each class */
    uint32_t max_long_segments[4];  /* bound on the segments of each class */
    uint32_t max_sublists[4];       /* bound on the sublists of each class */
    uint64_t bucket_bound[4];       /* largest bucket of the longest segment of each class */
    uint64_t off_status;            /* uint32 error flags raised by kernels (0 = none) */
    uint64_t workspace_bytes;       /* bytes these sizes need (<= the plan's workspace size) */
} dsort_seg_geometry_t;

int dsort_segmented_geometry(dsort_plan_t plan, uint64_t n, uint64_t num_segments,
                             uint64_t max_segment, dsort_seg_geometry_t *out);

/* Tuning of dsort_segmented's long segments, held by the plan.  classes = 0: one class with
 * the defaults (L = the largest tile, s = the smallest power of two that keeps every bucket
 * within one workgroup, Section 4's bound).  Otherwise class c (c < classes <= 4) holds lengths
 * in (upper[c-1], upper[c]] (strictly increasing; the last class also takes every longer
 * segment), with sublist_len[c] and samples[c] (0 = the defaults above).  Where a class's
 * (L, s) cannot bound the buckets of its longest segment in a call, that call uses the
 * defaults for the class.  Any tuning gives the same, unique, sorted result; it only changes
 * the speed. */
typedef struct {
    uint32_t classes;
    uint32_t from_cache;   /* set by dsort_autotune_segmented: 1 = read from its cache file */
    uint64_t upper[4];
    uint32_t sublist_len[4];
    uint32_t samples[4];
} dsort_seg_tuning_t;

/* Installs a tuning (NULL = the defaults).  Errors: DSORT_E_INVALID (bad plan, plan without
 * segments, or bounds not increasing), DSORT_E_UNSUPPORTED (an L that is not a power of two
 * in the tile range with at least 64 rows of items per thread, or an s that is not a power of
 * two up to min(L, 1024)), DSORT_E_CAPACITY (the plan's workspace is too small for it; every
 * tuning dsort_autotune_segmented can return fits). */
int dsort_set_seg_tuning(dsort_plan_t plan, const dsort_seg_tuning_t *tuning);
int dsort_get_seg_tuning(dsort_plan_t plan, dsort_seg_tuning_t *out);

/* Autotuner: times candidate tunings on the caller's batch and installs the fastest.  The
 * candidates for a set of lengths are the largest four tile lengths L (at least 64 rows of
 * items per thread) and, for each, the smallest admissible s and its double and quadruple.
 * (a) One class for all long segments: every candidate, timed on the whole batch, against the
 * defaults.  (b) Length classes split at small_capacity times 4, 16 and 64: every candidate of
 * a class timed on that class alone (the others at their defaults), the best per class
 * combined and timed on the whole batch.  The fastest whole-batch time of (a) and (b) wins.
 * Each run copies the batch (d_keys, d_values: left unchanged) into the caller's scratch
 * buffers (n keys, and n values for key/value plans) and sorts there, `repeats` times (at least
 * 1), timed with HIP events on `stream`.  Blocks until done.  Arguments as for dsort_segmented.
 * On success *out (may be NULL) receives the tuning; when the defaults win they are installed
 * as an explicit tuning with their (L, s) per class (no classes when no segment is long).
 * Persistence: if the environment variable DSORT_TUNE_CACHE names a file, a result is stored
 * there under (device: architecture, name and CU count; key type; values or not; segment class
 * = ceil(log2(max_segment))), and a later call with the same key installs the stored tuning
 * without timing anything (out->from_cache = 1) as long as it fits the plan.  The file is plain
 * text, rewritten through a temporary file and a rename; a write that fails only loses the
 * entry. */
int dsort_autotune_segmented(dsort_plan_t plan, const void *d_keys, const uint32_t *d_values,
                             uint64_t n, const uint64_t *d_offsets, uint64_t num_segments,
                             uint64_t max_segment, void *d_scratch_keys,
                             uint32_t *d_scratch_values, void *d_workspace, void *stream,
                             uint32_t repeats, dsort_seg_tuning_t *out);

/* ------------------------------------------------------------------------ served stream
 * A server sorts a stream of independent requests, each an array already in device memory
 * (caller-owned, sorted in place), as they arrive.  It owns a device arena of
 * `hbm_budget_bytes` (allocated at creation) from which every launch takes its workspace, and
 * `lanes` HIP streams (default priority) on which up to `lanes` launches overlap.  A background
 * thread forms the launches: when a lane is free it takes the oldest waiting request; requests
 * no longer than dsort_segmented's segment limit for their key layout are batched with the other
 * waiting ones of the same layout (key type and values or not) into one segmented sort (their
 * items are copied to a staging block of the arena and back); longer requests run alone as
 * dsort_keys/dsort_pairs would, in place.  A launch starts only if its requests' data plus its
 * workspace fit what is left of the budget, else the oldest request waits (first come, first
 * served), and at most `max_inflight` requests run at once.  Results are exactly those of dsort_keys/dsort_pairs on each request
 * alone.  The request's data must be complete in device memory when it is submitted (the
 * server's streams do not wait for other streams), and its buffers must stay valid and untouched
 * until dsort_poll reports it finished; two requests must not share memory. */
typedef struct dsort_server_s *dsort_server_t;

typedef struct {
    int key_type;        /* DSORT_U32 / DSORT_U64 / DSORT_F32 */
    int with_values;     /* 1: d_values holds n uint32 values (stable key/value sort) */
    void *d_keys;        /* n keys, device memory, natural alignment */
    uint32_t *d_values;  /* n values or NULL */
    uint64_t n;
} dsort_request_t;

typedef struct {
    int state;           /* 0 waiting, 1 running, 2 done, negative: failed with that status */
    int reserved;
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;  /* steady clock; 0 = not reached */
    uint64_t unit;       /* launch that ran it (requests of one batch share it) */
} dsort_result_t;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t units;              /* launches */
    uint64_t batched_units;      /* launches that sorted more than one request */
    uint64_t batched_requests;   /* requests sorted inside such launches */
    uint64_t max_batch;          /* most requests in one launch */
    uint64_t peak_arena_bytes;   /* most arena bytes in use at once */
    uint64_t peak_running_units; /* most launches on the device at once */
} dsort_server_stats_t;

/* Creates a server on the calling thread's current device.  lanes in 1..16; max_inflight >= 1
 * (also the most requests one batch holds, at most 4096).  Errors: DSORT_E_INVALID (budget
 * under 1 MiB, bad counts), DSORT_E_NOMEM (the arena could not be allocated), DSORT_E_HIP. */
int dsort_server_create(dsort_server_t *out, uint64_t hbm_budget_bytes, uint32_t max_inflight,
                        uint32_t lanes);
/* Queues a request and returns at once with its ticket.  Errors: DSORT_E_INVALID (bad type,
 * pointers or alignment), DSORT_E_CAPACITY (the request's data plus its workspace exceed the
 * budget, or it has no feasible plan). */
int dsort_submit(dsort_server_t server, const dsort_request_t *req, uint64_t *ticket);
/* Current state and timestamps of a ticket (never blocks).  DSORT_E_TICKET if unknown. */
int dsort_poll(dsort_server_t server, uint64_t ticket, dsort_result_t *out);
/* Forgets a finished ticket.  DSORT_E_INVALID if it is still waiting or running. */
int dsort_release(dsort_server_t server, uint64_t ticket);
int dsort_server_stats(dsort_server_t server, dsort_server_stats_t *out);
/* Waits for every queued and running request, then frees the server (NULL is accepted). */
int dsort_server_destroy(dsort_server_t server);

/* Per-kernel timing, for profiling.  dsort_set_timing(plan, 1) clears the record and makes
 * every later sorting call on `plan` bracket each kernel launch with two HIP events recorded
 * on the call's stream (events are created on first use and owned by the plan); 0 stops
 * recording.  After synchronising the stream(s) of the recorded calls, dsort_stage_times()
 * averages the recorded launches per stage: it writes up to `capacity` entries of `names`
 * (static strings, e.g. "s123_local_sort", "s9_bucket_sort"), `avg_ms` (mean milliseconds per
 * launch) and `launches` (launch count; each may be NULL), and the number of stages to *count.
 * Errors: DSORT_E_INVALID (bad plan, NULL count), DSORT_E_HIP (event query failed, e.g. the
 * work has not completed). */
int dsort_set_timing(dsort_plan_t plan, int enable);
int dsort_stage_times(dsort_plan_t plan, const char **names, float *avg_ms, uint32_t *launches,
                      int capacity, int *count);

#ifdef __cplusplus
}
#endif

#endif /* DSORT_H */
