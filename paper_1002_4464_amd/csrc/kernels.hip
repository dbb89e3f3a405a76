// HIP kernels for gfx950 (CDNA4, wave64) implementing Algorithm 1 of Dehne & Zaboli,
// "Deterministic Sample Sort For GPUs" (Section 4), and the host code that enqueues them.
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

namespace dsort {
namespace {

// ------------------------------------------------------------------------------ element types

struct C128 {  // 64-bit key with a 32-bit position (tie-break)
    uint64_t key;
    uint32_t pos;
    uint32_t unused;
};

__device__ __forceinline__ bool lt(uint32_t a, uint32_t b) { return a < b; }
__device__ __forceinline__ bool lt(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool lt(const C128 &a, const C128 &b) {
    return a.key < b.key || (a.key == b.key && a.pos < b.pos);
}

// Order used by the merge passes.  COMP: the elements are (key, position) composites whose
// positions increase with their initial LDS (or array) index, so inside a merge of two adjacent
// runs every position of the earlier run is below every position of the later one, and the
// composite order is the key order with ties going to the earlier run.  The merges take the
// earlier run on ties, so comparing keys alone gives the composite order.
template <class T, bool COMP> struct MergeLess {
    static __device__ __forceinline__ bool f(const T &a, const T &b) { return lt(a, b); }
};
template <> struct MergeLess<uint64_t, true> {  // (key << 32) | position
    static __device__ __forceinline__ bool f(uint64_t a, uint64_t b) {
        return (uint32_t)(a >> 32) < (uint32_t)(b >> 32);
    }
};
template <> struct MergeLess<C128, true> {
    static __device__ __forceinline__ bool f(const C128 &a, const C128 &b) { return a.key < b.key; }
};
template <bool COMP, class T> __device__ __forceinline__ bool mlt(const T &a, const T &b) {
    return MergeLess<T, COMP>::f(a, b);
}

// c ? a : b, field by field for the composite (a whole-struct select is lowered through
// scratch memory).
template <class T> __device__ __forceinline__ T sel(bool c, const T &a, const T &b) {
    return c ? a : b;
}
template <> __device__ __forceinline__ C128 sel<C128>(bool c, const C128 &a, const C128 &b) {
    C128 r;
    r.key = c ? a.key : b.key;
    r.pos = c ? a.pos : b.pos;
    r.unused = 0u;
    return r;
}

template <class T> struct MaxOf;
template <> struct MaxOf<uint32_t> {
    static __device__ __forceinline__ uint32_t get() { return 0xFFFFFFFFu; }
};
template <> struct MaxOf<uint64_t> {
    static __device__ __forceinline__ uint64_t get() { return ~0ull; }
};
template <> struct MaxOf<C128> {
    static __device__ __forceinline__ C128 get() { return C128{~0ull, 0xFFFFFFFFu, 0u}; }
};

// LDS index padding: one element of slack per 128 bytes, so that the blocked accesses of a
// wave (lane t touching t*E + k) spread over all banks.
template <class T> struct PadShift;
template <> struct PadShift<uint32_t> { static constexpr int v = 5; };
template <> struct PadShift<uint64_t> { static constexpr int v = 4; };
template <> struct PadShift<C128> { static constexpr int v = 3; };

template <class T> __device__ __forceinline__ uint32_t pidx(uint32_t i) {
    return i + (i >> PadShift<T>::v);
}
template <class T> constexpr uint32_t lds_elems(uint32_t cap) { return cap + (cap >> PadShift<T>::v); }


// f32 <-> IEEE totalOrder image.
__device__ __forceinline__ uint32_t f32_in(uint32_t b) {
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ uint32_t f32_out(uint32_t t) {
    return t ^ ((uint32_t)((int32_t)~t >> 31) | 0x80000000u);
}

// Per (key type, values) layout of the in-LDS sort element and of the sample composite.
// Key/value sorts carry the item's load position inside the tile as a tie-break, which makes
// every element distinct: any correct sorting network is then stable, and values are fetched
// by that position after the sort.
template <class K, bool V> struct Tr;

template <> struct Tr<uint32_t, false> {
    using K = uint32_t; using T = uint32_t; using SC = uint64_t;
    static __device__ __forceinline__ T make(K k, uint32_t) { return k; }
    static __device__ __forceinline__ K key(T e) { return e; }
    static __device__ __forceinline__ uint32_t lpos(T) { return 0; }
    static __device__ __forceinline__ T pad(uint32_t) { return 0xFFFFFFFFu; }
    static __device__ __forceinline__ SC samp(K k, uint32_t p) { return ((uint64_t)k << 32) | p; }
};
template <> struct Tr<uint32_t, true> {
    using K = uint32_t; using T = uint64_t; using SC = uint64_t;
    static __device__ __forceinline__ T make(K k, uint32_t p) { return ((uint64_t)k << 32) | p; }
    static __device__ __forceinline__ K key(T e) { return (uint32_t)(e >> 32); }
    static __device__ __forceinline__ uint32_t lpos(T e) { return (uint32_t)e; }
    static __device__ __forceinline__ T pad(uint32_t p) { return 0xFFFFFFFF00000000ull | p; }
    static __device__ __forceinline__ SC samp(K k, uint32_t p) { return ((uint64_t)k << 32) | p; }
};
template <> struct Tr<uint64_t, false> {
    using K = uint64_t; using T = uint64_t; using SC = C128;
    static __device__ __forceinline__ T make(K k, uint32_t) { return k; }
    static __device__ __forceinline__ K key(T e) { return e; }
    static __device__ __forceinline__ uint32_t lpos(T) { return 0; }
    static __device__ __forceinline__ T pad(uint32_t) { return ~0ull; }
    static __device__ __forceinline__ SC samp(K k, uint32_t p) { return C128{k, p, 0u}; }
};
template <> struct Tr<uint64_t, true> {
    using K = uint64_t; using T = C128; using SC = C128;
    static __device__ __forceinline__ T make(K k, uint32_t p) { return C128{k, p, 0u}; }
    static __device__ __forceinline__ K key(const T &e) { return e.key; }
    static __device__ __forceinline__ uint32_t lpos(const T &e) { return e.pos; }
    static __device__ __forceinline__ T pad(uint32_t p) { return C128{~0ull, p, 0u}; }
    static __device__ __forceinline__ SC samp(K k, uint32_t p) { return C128{k, p, 0u}; }
};

template <class K> struct KeyMax;
template <> struct KeyMax<uint32_t> { static constexpr uint32_t v = 0xFFFFFFFFu; };
template <> struct KeyMax<uint64_t> { static constexpr uint64_t v = ~0ull; };

// Position part i*L + r of a sample composite.
__device__ __forceinline__ uint32_t samp_pos(uint64_t c) { return (uint32_t)c; }
__device__ __forceinline__ uint32_t samp_pos(const C128 &c) { return c.pos; }

// Draw c of the SplitMix64 stream of `seed` (Steele, Lea and Flood 2014): the state after c + 1
// golden-ratio increments, through the published finaliser.  Randomized samples only.
__device__ __forceinline__ uint64_t splitmix64_draw(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------------------------ segments

// A set of segments (independent sort problems) and their partition into tiles of L items.
// seg == nullptr means one segment [0, n_single).
struct SegView {
    const uint4 *seg;          // {begin, size, ...} per segment
    const uint32_t *tile_off;  // G+1 entries: exclusive prefix of ceil(size/L) over segments
    uint32_t G;
    uint32_t n_single;
    uint32_t n_total;          // length of the keys array the segments index
    uint32_t max_tiles;        // capacity of the per-tile tables (tile_off views)
};

struct TileLoc {
    uint32_t g, i, seg_begin, seg_size, tile0, m;
    uint32_t piece0, pieces;  // the segment's piece table (bucket tables: {.., first piece, pieces})
};

__device__ __forceinline__ bool locate_tile(const SegView &sv, uint32_t L, uint32_t t,
                                            TileLoc &o) {
    if (!sv.tile_off) {
        const uint32_t m = (sv.n_single + L - 1) / L;
        if (t >= m) return false;
        o.g = 0; o.i = t; o.seg_begin = 0; o.seg_size = sv.n_single; o.tile0 = 0; o.m = m;
        o.piece0 = 0; o.pieces = 0;
        return true;
    }
    if (t >= sv.tile_off[sv.G] || sv.tile_off[sv.G] > sv.max_tiles) return false;
    uint32_t lo = 0, hi = sv.G;  // largest g with tile_off[g] <= t
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (sv.tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    o.g = lo;
    o.tile0 = sv.tile_off[lo];
    o.m = sv.tile_off[lo + 1] - o.tile0;
    o.i = t - o.tile0;
    const uint4 d = sv.seg[lo];
    o.seg_begin = d.x;
    o.seg_size = d.y;
    o.piece0 = d.z;
    o.pieces = d.w;
    // Defensive: tables written by earlier kernels must describe tiles inside the array.
    if ((uint64_t)d.x + d.y > sv.n_total || (uint64_t)o.i * L >= d.y) return false;
    return true;
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
    return x <= 1 ? 1u : 1u << (32 - __clz(x - 1));
}

// ------------------------------------------------------------------------------ block sort

template <class T> __device__ __forceinline__ void cmpx(T &a, T &b) {
    const bool sw = lt(b, a);
    const T lo = sel(sw, b, a);
    const T hi = sel(sw, a, b);
    a = lo;
    b = hi;
}

// Batcher's odd-even merge sort network over E registers: the network of the next power of
// two with every comparator that touches an index >= E left out (those indices would hold
// +infinity, which the network's low-to-high comparators never move).
template <class T, int E> __device__ __forceinline__ void reg_sort(T (&x)[E]) {
#pragma unroll
    for (int p = 1; p < E; p <<= 1)
#pragma unroll
        for (int k = p; k >= 1; k >>= 1)
#pragma unroll
            for (int j = k % p; j + k < E; j += 2 * k)
#pragma unroll
                for (int i = 0; i < k; ++i)
                    if (i + j + k < E && (i + j) / (2 * p) == (i + j + k) / (2 * p))
                        cmpx(x[i + j], x[i + j + k]);
}

// In-register merges of the sorted 16-item runs of 2, 4 and 8 neighbouring lanes into sorted
// runs of 32, 64 and 128 items (32-bit elements): Batcher's bitonic merge, the first half of it
// as compare-exchanges between lanes -- the partner's item comes through a DPP lane
// permutation, the lower lane keeps the minimum and the upper the maximum; the first stage of
// each merge pairs item e with the partner's item 15 - e, which merges two ascending runs
// without reversing one -- and its last four stages inside the lane.

// Eight compare-exchanges of one cross-lane stage: per item, v_sub_co_u32 with the partner's
// item as its DPP operand sets VCC where the partner's item is the smaller, s_xor flips that
// on the lanes that keep the minimum (`lower`), and v_cndmask (DPP operand again) keeps the own
// item where VCC is set, else takes the partner's: two vector instructions instead of min,
// max and a select.  The leading s_nop gives the DPP reads the two wait states a VGPR needs
// after a vector write; VCC and SCC (written by s_xor) are clobbered.
#define DS_XITEM(J, CTRL)                                                                   \
    "v_sub_co_u32_dpp %[t], vcc, %[s" #J "], %[x" #J "] " CTRL                             \
    " row_mask:0xf bank_mask:0xf\n\t"                                                       \
    "s_xor_b64 vcc, vcc, %[m]\n\t"                                                          \
    "v_cndmask_b32_dpp %[y" #J "], %[s" #J "], %[x" #J "], vcc " CTRL                      \
    " row_mask:0xf bank_mask:0xf\n\t"
#define DS_XCROSS8(CTRL)                                                                    \
    asm("s_nop 1\n\t" DS_XITEM(0, CTRL) DS_XITEM(1, CTRL) DS_XITEM(2, CTRL) DS_XITEM(3, CTRL) \
            DS_XITEM(4, CTRL) DS_XITEM(5, CTRL) DS_XITEM(6, CTRL) DS_XITEM(7, CTRL)         \
        : [y0] "=&v"(y[e0]), [y1] "=&v"(y[e0 + 1]), [y2] "=&v"(y[e0 + 2]),                 \
          [y3] "=&v"(y[e0 + 3]), [y4] "=&v"(y[e0 + 4]), [y5] "=&v"(y[e0 + 5]),             \
          [y6] "=&v"(y[e0 + 6]), [y7] "=&v"(y[e0 + 7]), [t] "=&v"(tmp)                     \
        : [s0] "v"(x[src(e0)]), [s1] "v"(x[src(e0 + 1)]), [s2] "v"(x[src(e0 + 2)]),        \
          [s3] "v"(x[src(e0 + 3)]), [s4] "v"(x[src(e0 + 4)]), [s5] "v"(x[src(e0 + 5)]),    \
          [s6] "v"(x[src(e0 + 6)]), [s7] "v"(x[src(e0 + 7)]), [x0] "v"(x[e0]),             \
          [x1] "v"(x[e0 + 1]), [x2] "v"(x[e0 + 2]), [x3] "v"(x[e0 + 3]), [x4] "v"(x[e0 + 4]), \
          [x5] "v"(x[e0 + 5]), [x6] "v"(x[e0 + 6]), [x7] "v"(x[e0 + 7]), [m] "s"(lower)    \
        : "vcc", "scc")

// The partner's item comes through a DPP lane permutation (CTRL); the lower lane of each pair
// keeps the minimum and the upper the maximum.  REV pairs item e with the partner's item 15 - e.
template <int CTRL, bool REV>
__device__ __forceinline__ void dpp_cross(uint32_t (&x)[16], uint64_t lower) {
    constexpr auto src = [](int e) { return REV ? 15 - e : e; };
    uint32_t y[16], tmp;
#pragma unroll
    for (int e0 = 0; e0 < 16; e0 += 8) {
        if constexpr (CTRL == 0xB1) DS_XCROSS8("quad_perm:[1,0,3,2]");
        else if constexpr (CTRL == 0x1B) DS_XCROSS8("quad_perm:[3,2,1,0]");
        else if constexpr (CTRL == 0x4E) DS_XCROSS8("quad_perm:[2,3,0,1]");
        else DS_XCROSS8("row_half_mirror");
    }
    (void)tmp;
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = y[e];
}
#undef DS_XCROSS8
#undef DS_XITEM

// Cross-lane stages whose minimum-keeping lanes fill whole DPP banks (groups of four lanes of
// a row): v_min writes those banks (bank mask LO) and v_max the others (HI), each reading the
// partner's item as its DPP operand (controls CL / CH), so the stage costs two vector
// instructions per item and no mask.  KIND 0: lane i of 8 against lane 7 - i (row_half_mirror),
// item e against item 15 - e; KIND 1: the same over 16 lanes (row_mirror); KIND 2: lane i
// against lane i ^ 4, item e against item e (the rotations by 12 and 4 lanes of a row bring
// lane i + 4 to the lower lanes and lane i - 4 to the upper ones).
#define DS_BITEM(J, CL, CH, LO, HI)                                                          \
    "v_min_u32_dpp %[y" #J "], %[s" #J "], %[x" #J "] " CL " row_mask:0xf bank_mask:" LO   \
    "\n\t"                                                                                   \
    "v_max_u32_dpp %[y" #J "], %[s" #J "], %[x" #J "] " CH " row_mask:0xf bank_mask:" HI   \
    "\n\t"
#define DS_BCROSS8(CL, CH, LO, HI)                                                            \
    asm("s_nop 1\n\t" DS_BITEM(0, CL, CH, LO, HI) DS_BITEM(1, CL, CH, LO, HI)                \
            DS_BITEM(2, CL, CH, LO, HI) DS_BITEM(3, CL, CH, LO, HI) DS_BITEM(4, CL, CH, LO, HI) \
                DS_BITEM(5, CL, CH, LO, HI) DS_BITEM(6, CL, CH, LO, HI)                       \
                    DS_BITEM(7, CL, CH, LO, HI)                                               \
        : [y0] "=&v"(y[e0]), [y1] "=&v"(y[e0 + 1]), [y2] "=&v"(y[e0 + 2]),                   \
          [y3] "=&v"(y[e0 + 3]), [y4] "=&v"(y[e0 + 4]), [y5] "=&v"(y[e0 + 5]),               \
          [y6] "=&v"(y[e0 + 6]), [y7] "=&v"(y[e0 + 7])                                       \
        : [s0] "v"(x[src(e0)]), [s1] "v"(x[src(e0 + 1)]), [s2] "v"(x[src(e0 + 2)]),          \
          [s3] "v"(x[src(e0 + 3)]), [s4] "v"(x[src(e0 + 4)]), [s5] "v"(x[src(e0 + 5)]),      \
          [s6] "v"(x[src(e0 + 6)]), [s7] "v"(x[src(e0 + 7)]), [x0] "v"(x[e0]),               \
          [x1] "v"(x[e0 + 1]), [x2] "v"(x[e0 + 2]), [x3] "v"(x[e0 + 3]), [x4] "v"(x[e0 + 4]), \
          [x5] "v"(x[e0 + 5]), [x6] "v"(x[e0 + 6]), [x7] "v"(x[e0 + 7]))

template <int KIND> __device__ __forceinline__ void dpp_cross_banks(uint32_t (&x)[16]) {
    constexpr auto src = [](int e) { return KIND >= 2 ? e : 15 - e; };
    uint32_t y[16];
#pragma unroll
    for (int e0 = 0; e0 < 16; e0 += 8) {
        if constexpr (KIND == 0) DS_BCROSS8("row_half_mirror", "row_half_mirror", "0x5", "0xa");
        else if constexpr (KIND == 1) DS_BCROSS8("row_mirror", "row_mirror", "0x3", "0xc");
        else if constexpr (KIND == 2) DS_BCROSS8("row_ror:12", "row_ror:4", "0x5", "0xa");
        else DS_BCROSS8("row_ror:8", "row_ror:8", "0x3", "0xc");  // lane i ^ 8
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = y[e];
}

// Stages whose partner lane lies in another row of 16, the partner's items brought by the LDS
// crossbar (no vector instruction) and the minimum kept by whole rows: row-masked v_min for
// the rows in LO, v_max for those in HI (the DPP control an identity).  KIND 0: lane i of 32
// against lane 31 - i, item e against item 15 - e (ds_swizzle reversal within 32 lanes, rows 0
// and 2 keep the minimum); KIND 1: lane i of 64 against lane 63 - i, item e against 15 - e
// (ds_bpermute; rows 0 and 1); KIND 2: lane i against lane i ^ 16, item e against item e
// (ds_swizzle; rows 0 and 2).
#define DS_RITEM(J, LO, HI)                                                                     \
    "v_min_u32_dpp %[y" #J "], %[p" #J "], %[x" #J "] quad_perm:[0,1,2,3] row_mask:" LO         \
    " bank_mask:0xf\n\t"                                                                        \
    "v_max_u32_dpp %[y" #J "], %[p" #J "], %[x" #J "] quad_perm:[0,1,2,3] row_mask:" HI         \
    " bank_mask:0xf\n\t"
#define DS_RCROSS8(LO, HI)                                                                      \
    asm("s_nop 1\n\t" DS_RITEM(0, LO, HI) DS_RITEM(1, LO, HI) DS_RITEM(2, LO, HI)               \
            DS_RITEM(3, LO, HI) DS_RITEM(4, LO, HI) DS_RITEM(5, LO, HI) DS_RITEM(6, LO, HI)     \
                DS_RITEM(7, LO, HI)                                                             \
        : [y0] "=&v"(y[e0]), [y1] "=&v"(y[e0 + 1]), [y2] "=&v"(y[e0 + 2]),                     \
          [y3] "=&v"(y[e0 + 3]), [y4] "=&v"(y[e0 + 4]), [y5] "=&v"(y[e0 + 5]),                 \
          [y6] "=&v"(y[e0 + 6]), [y7] "=&v"(y[e0 + 7])                                         \
        : [p0] "v"(p[0]), [p1] "v"(p[1]), [p2] "v"(p[2]), [p3] "v"(p[3]), [p4] "v"(p[4]),      \
          [p5] "v"(p[5]), [p6] "v"(p[6]), [p7] "v"(p[7]), [x0] "v"(x[e0]),                     \
          [x1] "v"(x[e0 + 1]), [x2] "v"(x[e0 + 2]), [x3] "v"(x[e0 + 3]), [x4] "v"(x[e0 + 4]),   \
          [x5] "v"(x[e0 + 5]), [x6] "v"(x[e0 + 6]), [x7] "v"(x[e0 + 7]))
template <int KIND> __device__ __forceinline__ void cross_rows(uint32_t (&x)[16]) {
    const int rev_addr = (int)(63 - (threadIdx.x & 63)) * 4;  // ds_bpermute source lane, bytes
    uint32_t y[16];
#pragma unroll
    for (int e0 = 0; e0 < 16; e0 += 8) {
        uint32_t p[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int v = (int)x[KIND == 2 ? e0 + j : 15 - e0 - j];
            p[j] = (uint32_t)(KIND == 0   ? __builtin_amdgcn_ds_swizzle(v, 0x7C1F)
                              : KIND == 1 ? __builtin_amdgcn_ds_bpermute(rev_addr, v)
                                          : __builtin_amdgcn_ds_swizzle(v, 0x401F));
        }
        if constexpr (KIND == 1) DS_RCROSS8("0x3", "0xc");
        else DS_RCROSS8("0x5", "0xa");
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = y[e];
}
#undef DS_RCROSS8
#undef DS_RITEM
#undef DS_BCROSS8
#undef DS_BITEM

__device__ __forceinline__ void inlane_bitonic(uint32_t (&x)[16]) {
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            if ((e & d) == 0) {
                const uint32_t a = x[e], b = x[e | d];
                x[e] = min(a, b);
                x[e | d] = max(a, b);
            }
}

// DPP controls: quad_perm [1,0,3,2], [3,2,1,0], [2,3,0,1] and row_half_mirror (lane i of
// each 8 reads lane 7 - i).
constexpr int kDppSwap1 = 0xB1, kDppRev4 = 0x1B, kDppSwap2 = 0x4E, kDppRev8 = 0x141;

// lanes whose bit 0 or 1 is clear: the lower lane of a pair 1 or 2 lanes apart
constexpr uint64_t kLow1 = 0x5555555555555555ull, kLow2 = 0x3333333333333333ull;

__device__ __forceinline__ void dpp_merge_128(uint32_t (&x)[16]) {
    dpp_cross<kDppSwap1, true>(x, kLow1);
    inlane_bitonic(x);
    dpp_cross<kDppRev4, true>(x, kLow2);
    dpp_cross<kDppSwap1, false>(x, kLow1);
    inlane_bitonic(x);
    dpp_cross_banks<0>(x);
    dpp_cross<kDppSwap2, false>(x, kLow2);
    dpp_cross<kDppSwap1, false>(x, kLow1);
    inlane_bitonic(x);
}

// The next merge, of the sorted 128-item runs of the two halves of a 16-lane row into one run
// of 256 items.
__device__ __forceinline__ void dpp_merge_256(uint32_t (&x)[16]) {
    dpp_cross_banks<1>(x);
    dpp_cross_banks<2>(x);
    dpp_cross<kDppSwap2, false>(x, kLow2);
    dpp_cross<kDppSwap1, false>(x, kLow1);
    inlane_bitonic(x);
}

// And the next, of the 256-item runs of two neighbouring rows into one run of 512 items.
__device__ __forceinline__ void dpp_merge_512(uint32_t (&x)[16]) {
    cross_rows<0>(x);
    dpp_cross_banks<3>(x);
    dpp_cross_banks<2>(x);
    dpp_cross<kDppSwap2, false>(x, kLow2);
    dpp_cross<kDppSwap1, false>(x, kLow1);
    inlane_bitonic(x);
}

// And the last, of the 512-item runs of the two halves of a wave into one run of 1024 items.
__device__ __forceinline__ void dpp_merge_1024(uint32_t (&x)[16]) {
    cross_rows<1>(x);
    cross_rows<2>(x);
    dpp_cross_banks<3>(x);
    dpp_cross_banks<2>(x);
    dpp_cross<kDppSwap2, false>(x, kLow2);
    dpp_cross<kDppSwap1, false>(x, kLow1);
    inlane_bitonic(x);
}

// Byte offset of padded LDS element i: (i + (i >> shift)) << log2(sizeof(T)) as one
// v_add_lshl_u32 (the compiler otherwise splits the scaling into three instructions).
template <class T> struct SizeLog2;
template <> struct SizeLog2<uint32_t> { static constexpr int v = 2; };
template <> struct SizeLog2<uint64_t> { static constexpr int v = 3; };
template <> struct SizeLog2<C128> { static constexpr int v = 4; };

#define DS_LDS __attribute__((address_space(3)))

template <class T> __device__ __forceinline__ T lds_load(const DS_LDS T *p) { return *p; }
template <> __device__ __forceinline__ C128 lds_load<C128>(const DS_LDS C128 *p) {
    return C128{p->key, p->pos, 0u};
}

template <class T> __device__ __forceinline__ T lds_at(const T *lds, uint32_t i) {
    uint32_t off;
    asm("v_add_lshl_u32 %0, %1, %2, %3"
        : "=v"(off)
        : "v"(i), "v"(i >> PadShift<T>::v), "i"(SizeLog2<T>::v));
    const DS_LDS char *base = (const DS_LDS char *)lds;
    return lds_load<T>((const DS_LDS T *)(base + off));
}

// Values of key/value sorts after the sort: once a sorted element's key has been written out,
// the key half of its LDS slot (u32 keys: the high word of (key << 32) | position; u64 keys:
// the unused word of the 16-byte element) holds the value whose load position is that slot's
// index, while the position half still names the slot of the element's own value.
template <class T> struct ValSlot;
template <> struct ValSlot<uint64_t> {
    static constexpr int val_word = 1, pos_word = 0, words = 2;
};
template <> struct ValSlot<C128> {
    static constexpr int val_word = 3, pos_word = 2, words = 4;
};
template <class T> __device__ __forceinline__ void put_val(T *lds, uint32_t i, uint32_t v) {
    ((uint32_t *)(lds + pidx<T>(i)))[ValSlot<T>::val_word] = v;
}
template <class T> __device__ __forceinline__ uint32_t val_of_sorted(const T *lds, uint32_t x) {
    const uint32_t p = ((const uint32_t *)(lds + pidx<T>(x)))[ValSlot<T>::pos_word];
    return ((const uint32_t *)(lds + pidx<T>(p)))[ValSlot<T>::val_word];
}

// Merge path: number of A items among the first `diag` outputs of the stable merge of
// A = lds[a0, a0+na) and B = lds[b0, b0+nb) (A wins ties).
template <class T, bool COMP = false>
__device__ __forceinline__ uint32_t merge_path(const T *lds, uint32_t a0, uint32_t na,
                                               uint32_t b0, uint32_t nb, uint32_t diag) {
    uint32_t lo = diag > nb ? diag - nb : 0;
    uint32_t hi = diag < na ? diag : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const T av = lds_at<T>(lds, a0 + mid);
        const T bv = lds_at<T>(lds, b0 + diag - 1 - mid);
        if (mlt<COMP>(bv, av)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// The same split found with a fixed number of halving steps, top = a power of two >= na and
// >= nb (the same for every lane, so the loop needs no exit test): the largest a in [lo, hi]
// whose A[a - 1] does not follow B[diag - a], stepping from lo by top, top / 2, ..., 1 with
// each probe clamped to hi (the first probe is hi itself).  Every probe reads inside A and B.
template <class T, bool COMP = false>
__device__ __forceinline__ uint32_t merge_split(const T *lds, uint32_t a0, uint32_t na,
                                                uint32_t b0, uint32_t nb, uint32_t diag,
                                                uint32_t top) {
    const uint32_t lo = diag > nb ? diag - nb : 0, hi = min(diag, na);
    uint32_t pos = lo;
    if (lo < hi) {
        const uint32_t am1 = a0 - 1, bd = b0 + diag;
        for (uint32_t step = top; step; step >>= 1) {
            const uint32_t q = min(pos + step, hi);
            const T av = lds_at<T>(lds, am1 + q);
            const T bv = lds_at<T>(lds, bd - q);
            pos = mlt<COMP>(bv, av) ? pos : q;
        }
    }
    return pos;
}

// Serial stable merge of E outputs starting at A index ai (< a_end) / B index bi (< b_end),
// for an LDS array with one readable element past every index it can reach (so no clamp).
// ai and bi are left at the next unmerged items.
template <class T, int E, bool COMP = false>
__device__ __forceinline__ void serial_merge_nc(const T *lds, uint32_t &ai, uint32_t a_end,
                                                uint32_t &bi, uint32_t b_end, T (&out)[E]) {
    T av = lds_at<T>(lds, ai);
    T bv = lds_at<T>(lds, bi);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const bool take_a = (bi >= b_end) || ((ai < a_end) && !mlt<COMP>(bv, av));
        out[k] = sel(take_a, av, bv);
        ai += take_a ? 1u : 0u;
        bi += take_a ? 0u : 1u;
        const T v = lds_at<T>(lds, take_a ? ai : bi);
        av = sel(take_a, v, av);
        bv = sel(take_a, bv, v);
    }
}

// Serial stable merge of E outputs starting at A index ai (< a_end) / B index bi (< b_end).
// `lim` is any valid LDS index used to keep speculative reads in bounds.
template <class T, int E, bool COMP = false>
__device__ __forceinline__ void serial_merge(const T *lds, uint32_t ai, uint32_t a_end,
                                             uint32_t bi, uint32_t b_end, uint32_t lim,
                                             T (&out)[E]) {
    T av = lds[pidx<T>(min(ai, lim))];
    T bv = lds[pidx<T>(min(bi, lim))];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const bool take_a = (bi >= b_end) || ((ai < a_end) && !mlt<COMP>(bv, av));
        out[k] = sel(take_a, av, bv);
        const uint32_t nxt = take_a ? ai + 1 : bi + 1;
        ai = take_a ? ai + 1 : ai;
        bi = take_a ? bi : bi + 1;
        const T v = lds[pidx<T>(min(nxt, lim))];
        av = sel(take_a, v, av);
        bv = sel(take_a, bv, v);
    }
}

// Sorts lds[0, P) in place (P a multiple of E, E <= P <= E * blockDim.x; lds must hold
// lds_elems(P) + 1 elements, the last one only ever read speculatively).  Thread t owns
// items [tE, tE+E): a register network sorts them, then merge passes double the sorted run
// length (runs of E * 2^lv items); when P / E is not a power of two the last run of a pass is
// shorter (or has no partner).  32-bit elements with E = 16 and P a multiple of 128 merge
// their first three passes in registers across lanes (dpp_merge_128), the fourth too when P
// is a multiple of 256 (dpp_merge_256), the fifth when it is one of 512 (dpp_merge_512) and
// the sixth, across whole waves, when it is one of 1024 (dpp_merge_1024).  R0 > E: lds already
// holds sorted runs of R0 items (R0 a power of two times E), so sorting starts with the
// merge pass of those runs.
// All threads of the block must call it.  COMP: see MergeLess (the register network always
// compares whole elements; only the merges may compare keys alone).  TWO: when P is a multiple
// of 2E, every LDS merge pass gives each active thread two consecutive blocks of E outputs, so
// one split search serves 2E outputs (measured on the 16K-item tile sorts: 8 % fewer VALU
// instructions; slower in the bucket kernels, whose register count it raises past 64).
template <class T, int E, bool COMP = false, bool TWO = false>
__device__ __forceinline__ void block_sort(T *lds, uint32_t P, uint32_t R0 = E) {
    const uint32_t t = threadIdx.x;
    const bool act = t * E < P;
    // whole 8-lane groups: every lane whose partners it reads is active with it
    const bool dpp = R0 <= E && sizeof(T) == 4 && E == 16 && P % 128 == 0;
    const bool dpp16 = dpp && P % 256 == 0;  // whole 16-lane rows: one more register merge
    const bool dpp32 = dpp && P % 512 == 0;  // whole 32-lane halves: and another
    const bool dpp64 = dpp && P % 1024 == 0;  // whole waves: and one more
    T x[E];
    if (R0 <= E && act) {
#pragma unroll
        for (int k = 0; k < E; ++k) x[k] = lds[pidx<T>(t * E + k)];
        reg_sort<T, E>(x);
        if constexpr (sizeof(T) == 4 && E == 16) {
            if (dpp) dpp_merge_128(x);
            if (dpp16) dpp_merge_256(x);
            if (dpp32) dpp_merge_512(x);
            if (dpp64) dpp_merge_1024(x);
        }
#pragma unroll
        for (int k = 0; k < E; ++k) lds[pidx<T>(t * E + k)] = x[k];
    }
    const uint32_t Rs = R0 > E         ? R0
                        : dpp64   ? 64 * E
                        : dpp32   ? 32 * E
                        : dpp16   ? 16 * E
                        : dpp     ? 8 * E
                                  : E;
    for (uint32_t R = Rs, pair = 2 * Rs / E, top = pow2_at_least(Rs); R < P;
         R <<= 1, pair <<= 1, top <<= 1) {
        __syncthreads();
        if (TWO && P % (2 * E) == 0) {
            // every pair holds a multiple of 2E items, so a thread's 2E outputs share one pair
            T y[E];
            const bool act2 = t * 2 * E < P;
            if (act2) {
                const uint32_t start = t * 2 * E;
                const uint32_t base = start & ~(2 * R - 1);  // first item of the run pair
                const uint32_t diag = start - base;
                const uint32_t na = min(R, P - base);
                const uint32_t nb = min(R, P - base - na);
                const uint32_t a = merge_split<T, COMP>(lds, base, na, base + na, nb, diag, top);
                uint32_t ai = base + a, bi = base + na + diag - a;
                serial_merge_nc<T, E, COMP>(lds, ai, base + na, bi, base + na + nb, x);
                serial_merge_nc<T, E, COMP>(lds, ai, base + na, bi, base + na + nb, y);
            }
            __syncthreads();
            if (act2) {
#pragma unroll
                for (int k = 0; k < E; ++k) lds[pidx<T>(t * 2 * E + k)] = x[k];
#pragma unroll
                for (int k = 0; k < E; ++k) lds[pidx<T>(t * 2 * E + E + k)] = y[k];
            }
            continue;
        }
        if (act) {
            const uint32_t start = t * E;
            const uint32_t base = (t & ~(pair - 1)) * E;  // first item of the thread's run pair
            const uint32_t diag = start - base;
            const uint32_t na = min(R, P - base);
            const uint32_t nb = min(R, P - base - na);
            const uint32_t a = merge_split<T, COMP>(lds, base, na, base + na, nb, diag, top);
            uint32_t ai = base + a, bi = base + na + diag - a;
            serial_merge_nc<T, E, COMP>(lds, ai, base + na, bi, base + na + nb, x);
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < E; ++k) lds[pidx<T>(t * E + k)] = x[k];
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------ wave and block scans

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts by 1, 2, 4, 8 within
// each row of 16 lanes, then row broadcasts of lane 15 (into rows 1, 3) and lane 31 (rows 2, 3).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false); // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false); // row_bcast:31
    return x;
}

// Exclusive scan of one value per thread over the block (blockDim a multiple of 64, at most
// 1024); *total receives the block sum.  wsum: LDS scratch of 17 words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *wsum, uint32_t &total) {
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        const uint32_t v = lane < nw ? wsum[lane] : 0u;
        const uint32_t vi = wave_incl_scan(v);
        if (lane < nw) wsum[lane] = vi - v;
        if (lane == nw - 1) wsum[16] = vi;
    }
    __syncthreads();
    total = wsum[16];
    return wsum[w] + inc - x;
}


// ------------------------------------------------------------------------------ Steps 1-3, 9

enum { MODE_SAMPLE = 0, MODE_FINAL = 1 };

struct TileArgs {
    const void *src_keys;
    void *dst_keys;
    const uint32_t *src_vals;
    uint32_t *dst_vals;
    SegView sv;
    uint32_t L;      // MODE_SAMPLE: sublist length
    uint32_t s;      // MODE_SAMPLE: samples per sublist
    void *samples;   // MODE_SAMPLE: m*s composites, row = global tile index
    uint32_t *status;
    const uint32_t *pdst;  // GIN: bucket-major destinations l_ij of the previous level's pieces
    const uint32_t *psrc;  // GIN: their source positions in src_keys / src_vals
    uint64_t seed;         // MODE_SAMPLE without GIN, random != 0: the samples' stream seed
    uint32_t random;       // 1: Step 3 takes s random sorted positions instead of chunk ends
};

// Sublists of a second level read straight from the pieces of the first (Step 8 of the first
// level fused into Step 1 of the second): item x of a level-1 bucket is item x - l_ij of the
// piece A_ij with l_ij <= x < l_(i+1)j.  The pieces that cover one tile are staged in LDS
// kTilePieces at a time; each wave streams its share of the chunk's items, every lane
// following the piece its item is in, and `store(x, source index)` puts item x in place.
constexpr uint32_t kTilePieces = 1024;

// Largest p < np with pdst[p] - base <= x (pdst[0] - base is 0 for a bucket's first piece).
// Wave-cooperative search over global memory: the nl lanes of the (whole) wave probe nl
// evenly spaced positions at once, cutting the range nl + 1 ways per round; every lane
// returns the answer.
__device__ __forceinline__ uint32_t wave_piece_search(const uint32_t *pdst, uint32_t np,
                                                      uint32_t base, uint32_t x) {
    const uint32_t nl = min(64u, blockDim.x), lane = threadIdx.x & (nl - 1);
    uint32_t lo = 0, hi = np;  // pdst[lo] qualifies; the answer lies in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + nl) / (nl + 1);
        const uint32_t p = lo + (lane + 1) * step;
        const bool ok = p < hi && pdst[p] - base <= x;
        const uint64_t mask = __ballot(ok);  // the qualifying probes are a prefix of the lanes
        lo += (mask ? 64u - (uint32_t)__clzll(mask) : 0u) * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

template <class F>
__device__ __forceinline__ void tile_gather(const uint32_t *pdst, const uint32_t *psrc,
                                            uint32_t bucket_begin, uint32_t x0, uint32_t count,
                                            uint32_t p_first, uint32_t p_last, uint32_t *tb,
                                            uint32_t *sb, F store) {
    // lanes per wave (blocks of fewer than 64 threads are one partial wave)
    const uint32_t wl = min(64u, blockDim.x), tid = threadIdx.x;
    const uint32_t lane = tid & (wl - 1), w = tid / wl, nw = blockDim.x / wl;
    for (uint32_t c = p_first; c <= p_last; c += kTilePieces) {
        const uint32_t nk = min(kTilePieces, p_last + 1 - c);
        __syncthreads();  // the previous chunk (or caller) is done with tb / sb
        for (uint32_t k = tid; k <= nk; k += blockDim.x) {
            uint32_t b = count;  // the tile's end closes the last piece
            if (c + k <= p_last) {
                const uint32_t at = pdst[c + k] - bucket_begin;  // offset in the bucket
                b = min(max(at, x0) - x0, count);
                if (k < nk) sb[k] = psrc[c + k] - at + x0;  // + x: source of tile item x
            }
            tb[k] = b;
        }
        __syncthreads();
        const uint32_t lo = tb[0], hi = tb[nk];
        const uint32_t span = ((hi - lo + nw - 1) / nw + wl - 1) / wl * wl;
        const uint32_t xs = lo + w * span, xe = min(hi, xs + span);
        if (xs >= xe) continue;
        uint32_t p = 0;
        {
            uint32_t l = 0, h = nk - 1;  // largest k with tb[k] <= item
            const uint32_t xi = min(xs + lane, xe - 1);
            while (l < h) {
                const uint32_t mid = (l + h + 1) >> 1;
                if (tb[mid] <= xi) l = mid; else h = mid - 1;
            }
            p = l;
        }
        for (uint32_t row = xs; row < xe; row += 4 * wl) {
            uint32_t si[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t xu = row + wl * u + lane;
                if (xu < xe) {
                    while (xu >= tb[p + 1]) ++p;
                    si[u] = sb[p] + xu;
                }
            }
            store.template run<4>(row + lane, wl, xe, si);
        }
    }
}

// Stores of tile_gather: keys into the LDS sort array (as elements carrying their tile
// position), values into the slots' free halves (put_val).  Source indices past the array are
// never read.
template <class K, class R, class T> struct GatherKeys {
    const K *src;
    T *lds;
    uint32_t n_total;
    // items x0 + stride * u (u < U) below xe come from source indices si[u]
    template <int U>
    __device__ __forceinline__ void run(uint32_t x0, uint32_t stride, uint32_t xe,
                                        const uint32_t (&si)[U]) const {
        K v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t xu = x0 + stride * u;
            v[u] = (xu < xe && si[u] < n_total) ? src[si[u]] : KeyMax<K>::v;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t xu = x0 + stride * u;
            if (xu < xe) lds[pidx<T>(xu)] = R::make(v[u], xu);
        }
    }
};
template <class T> struct GatherVals {
    const uint32_t *src;
    T *lds;
    uint32_t n_total;
    template <int U>
    __device__ __forceinline__ void run(uint32_t x0, uint32_t stride, uint32_t xe,
                                        const uint32_t (&si)[U]) const {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t xu = x0 + stride * u;
            v[u] = (xu < xe && si[u] < n_total) ? src[si[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t xu = x0 + stride * u;
            if (xu < xe) put_val<T>(lds, xu, v[u]);
        }
    }
};

// MODE_SAMPLE (Steps 1-3): one workgroup per sublist of L items; writes the sorted sublist in
// place and its s samples.  MODE_FINAL (Step 9): one workgroup per segment of at most CAP
// items, sorted from src into dst (which may alias).  XIN/XOUT apply the f32 order map.
// GIN (MODE_SAMPLE, second level): the sublist is gathered from the previous level's pieces
// (see tile_gather) and the sorted sublist goes to dst, which must not alias src.
template <class K, bool V, int E, int CAP, int MODE, bool XIN, bool XOUT, bool GIN = false>
__global__ __launch_bounds__(CAP / E) void k_tile(TileArgs a) {
    using R = Tr<K, V>;
    using T = typename R::T;
    static_assert(!GIN || (MODE == MODE_SAMPLE && !XIN), "piece gathers feed Steps 1-3 only");
    __shared__ T lds[lds_elems<T>(CAP) + 1];
    __shared__ uint32_t tb[GIN ? kTilePieces + 1 : 1], sb[GIN ? kTilePieces : 1], pr[2];
    constexpr bool kCanRandom = MODE == MODE_SAMPLE && !GIN;
    __shared__ uint32_t rp[kCanRandom ? 1024 : 1];  // randomized samples: (position, k) keys
    const uint32_t tid = threadIdx.x;
    const uint32_t bd = blockDim.x;

    uint32_t begin, count, P;
    TileLoc loc{};
    if (MODE == MODE_SAMPLE) {
        if (!locate_tile(a.sv, a.L, blockIdx.x, loc)) return;
        begin = loc.seg_begin + loc.i * a.L;
        count = min(a.L, loc.seg_size - loc.i * a.L);
        P = a.L;
    } else {
        uint4 d = a.sv.seg ? a.sv.seg[blockIdx.x] : make_uint4(0u, a.sv.n_single, 0u, 0u);
        begin = d.x;
        count = d.y;
        if (count == 0) return;
        if (count > CAP || (uint64_t)begin + count > a.sv.n_total) {
            if (tid == 0) atomicOr(a.status, 1u);
            return;
        }
        P = max((uint32_t)E, pow2_at_least(count));
    }

    const K *src = (const K *)a.src_keys;
    uint32_t p_first = 0, p_last = 0;
    if (GIN) {
        // pieces holding the tile's first and last items (one wave each, or one wave both)
        const uint32_t wl = min(64u, bd);
        for (uint32_t q = tid / wl; q < 2; q += bd / wl) {
            const uint32_t x = loc.i * a.L + (q == 0 ? 0u : count - 1);
            const uint32_t p = wave_piece_search(a.pdst + loc.piece0, loc.pieces, loc.seg_begin, x);
            if ((tid & (wl - 1)) == 0) pr[q] = p;
        }
        __syncthreads();
        p_first = pr[0];
        p_last = pr[1];
        tile_gather(a.pdst + loc.piece0, a.psrc + loc.piece0, loc.seg_begin, loc.i * a.L, count,
                    p_first, p_last, tb, sb, GatherKeys<K, R, T>{src, lds, a.sv.n_total});
        for (uint32_t i = count + tid; i < P; i += bd) lds[pidx<T>(i)] = R::pad(i);
    } else {
        for (uint32_t i = tid; i < P; i += bd) {
            T e;
            if (i < count) {
                K k = src[begin + i];
                if (XIN) k = (K)f32_in((uint32_t)k);
                e = R::make(k, i);
            } else {
                e = R::pad(i);
            }
            lds[pidx<T>(i)] = e;
        }
    }
    __syncthreads();
    // key/value elements carry their load position
    block_sort<T, E, V, sizeof(T) == 4 && E == 16>(lds, P);

    if (MODE == MODE_SAMPLE) {
        typename R::SC *smp = (typename R::SC *)a.samples + (size_t)(loc.tile0 + loc.i) * a.s;
        if (kCanRandom && a.random) {
            // Randomized variant: sample k sits at sorted position ((d >> 32) * L) >> 32, d the
            // draw i*s + k.  The samples are written in position order (ties by k), so that each
            // sublist's samples stay a sorted run for Step 4 and for the rank bisection.
            for (uint32_t k = tid; k < a.s; k += bd) {
                const uint64_t d = splitmix64_draw(a.seed, (uint64_t)loc.i * a.s + k);
                rp[k] = (__umulhi((uint32_t)(d >> 32), a.L) << 10) | k;  // L <= 2^16, s <= 2^10
            }
            __syncthreads();
            for (uint32_t k = tid; k < a.s; k += bd) {
                const uint32_t me = rp[k];
                uint32_t rank = 0;
                for (uint32_t q = 0; q < a.s; ++q) rank += rp[q] < me ? 1u : 0u;
                const uint32_t r = me >> 10;
                smp[rank] = R::samp(R::key(lds[pidx<T>(r)]), loc.i * a.L + r);
            }
        } else {
            const uint32_t w = a.L / a.s;
            for (uint32_t k = tid; k < a.s; k += bd) {
                const uint32_t r = (k + 1) * w - 1;
                smp[k] = R::samp(R::key(lds[pidx<T>(r)]), loc.i * a.L + r);
            }
        }
    }

    K *dst = (K *)a.dst_keys;
#pragma unroll 2
    for (int q = 0; q < E; ++q) {
        const uint32_t i = tid + q * bd;
        if (i < count) {
            K k = R::key(lds[pidx<T>(i)]);
            if (XOUT) k = (K)f32_out((uint32_t)k);
            dst[begin + i] = k;
        }
    }
    if constexpr (V) {
        __syncthreads();
        if (GIN)
            tile_gather(a.pdst + loc.piece0, a.psrc + loc.piece0, loc.seg_begin, loc.i * a.L,
                        count, p_first, p_last, tb, sb,
                        GatherVals<T>{a.src_vals, lds, a.sv.n_total});
        else
            for (uint32_t i = tid; i < count; i += bd) put_val<T>(lds, i, a.src_vals[begin + i]);
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * bd;
            if (i < count) a.dst_vals[begin + i] = val_of_sorted<T>(lds, i);
        }
    }
}

// ------------------------------------------------------------------------------ Step 4

// Sorts one range of sample composites inside one workgroup: per segment (the samples of
// segment g are rows tile_off[g] .. tile_off[g+1]-1, s per row) or per fixed chunk.
template <class SC, int E, int CAP>
__global__ __launch_bounds__(CAP / E) void k_sort_samples(const SC *src, SC *dst, SegView sv,
                                                          uint32_t L, uint32_t s,
                                                          uint32_t chunk_total,
                                                          uint32_t *status) {
    __shared__ SC lds[lds_elems<SC>(CAP) + 1];
    const uint32_t tid = threadIdx.x;
    uint32_t begin, count;
    if (chunk_total) {  // fixed chunks of CAP
        begin = blockIdx.x * CAP;
        if (begin >= chunk_total) return;
        count = min((uint32_t)CAP, chunk_total - begin);
    } else if (!sv.tile_off) {
        begin = 0;
        count = ((sv.n_single + L - 1) / L) * s;
    } else {
        if (sv.tile_off[blockIdx.x + 1] > sv.max_tiles) {
            if (tid == 0) atomicOr(status, 4u);
            return;
        }
        begin = sv.tile_off[blockIdx.x] * s;
        count = sv.tile_off[blockIdx.x + 1] * s - begin;
    }
    if (count == 0) return;
    if (count > CAP) {
        if (tid == 0) atomicOr(status, 2u);
        return;
    }
    const uint32_t P = max((uint32_t)E, pow2_at_least(count));
    for (uint32_t i = tid; i < P; i += blockDim.x)
        lds[pidx<SC>(i)] = i < count ? src[begin + i] : MaxOf<SC>::get();
    __syncthreads();
    // Each sublist's s samples are already in order (they come from its sorted items) and
    // every range starts on a row, so the sort starts from runs of s; sample composites are
    // in position order.
    block_sort<SC, E, true>(lds, P, s > (uint32_t)E ? s : (uint32_t)E);
    for (uint32_t i = tid; i < count; i += blockDim.x) dst[begin + i] = lds[pidx<SC>(i)];
}

// One round of a global merge sort over sorted runs of length R (R a multiple of CAP):
// workgroup b writes outputs [b*CAP, (b+1)*CAP) of the merge of its run pair (merged in
// registers, staged back in LDS, stored with consecutive lanes on consecutive items).
template <class SC, int E, int CAP>
__global__ __launch_bounds__(CAP / E) void k_merge_round(const SC *src, SC *dst, uint32_t total,
                                                         uint32_t R) {
    __shared__ SC lds[lds_elems<SC>(CAP)];
    __shared__ uint32_t split[2];
    const uint32_t tid = threadIdx.x;
    const uint32_t c0 = blockIdx.x * CAP;
    if (c0 >= total) return;
    const uint32_t pb = c0 & ~(2 * R - 1);
    const uint32_t a0 = pb, a1 = min(pb + R, total);
    const uint32_t b0 = a1, b1 = min(pb + 2 * R, total);
    const uint32_t na = a1 - a0, nb = b1 - b0;
    const uint32_t d0 = c0 - pb, d1 = min(d0 + CAP, na + nb);
    if (tid < 128) {  // wave 0 finds the split of d0, wave 1 that of d1, 64 probes per round
        const uint32_t lane = tid & 63;
        const uint32_t d = (tid >> 6) ? d1 : d0;
        uint32_t lo = d > nb ? d - nb : 0, hi = min(d, na);
        while (lo < hi) {  // smallest x in [lo, hi) with B[d-1-x] < A[x], else hi
            const uint32_t step = (hi - lo + 63) >> 6;
            const uint32_t x = lo + lane * step;
            const bool pr = x >= hi || mlt<true>(src[b0 + d - 1 - x], src[a0 + x]);
            const uint64_t m = __ballot(pr);
            if (m == 0) {
                lo = lo + 63 * step + 1;
            } else {
                const uint32_t f = (uint32_t)__builtin_ctzll(m);
                const uint32_t nh = min(lo + f * step, hi);
                lo = f ? lo + (f - 1) * step + 1 : lo;
                hi = nh;
            }
        }
        if (lane == 0) split[tid >> 6] = lo;
    }
    __syncthreads();
    const uint32_t ia = a0 + split[0], la = split[1] - split[0];
    const uint32_t ib = b0 + (d0 - split[0]), lb = (d1 - d0) - la;
    for (uint32_t i = tid; i < la + lb; i += blockDim.x)
        lds[pidx<SC>(i)] = i < la ? src[ia + i] : src[ib + i - la];
    __syncthreads();
    const uint32_t diag = tid * E;
    const uint32_t tot = la + lb;
    SC out[E];
    if (diag < tot) {
        const uint32_t x = merge_path<SC, true>(lds, 0, la, la, lb, diag);
        serial_merge<SC, E, true>(lds, x, la, la + diag - x, tot, tot - 1, out);
    }
    __syncthreads();  // back through LDS, so that the stores below are coalesced
    if (diag < tot) {
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (diag + k < tot) lds[pidx<SC>(diag + k)] = out[k];
    }
    __syncthreads();
    for (uint32_t i = tid; i < tot; i += blockDim.x) dst[c0 + i] = lds[pidx<SC>(i)];
}

// ------------------------------------------------------------------------------ Steps 5-6

// One workgroup per sublist; it locates every global sample g_j = S[(j+1) m - 1] of the
// sublist's segment: r_ij = #{x : (A_i[x], i*L + x) <= g_j}, a monotone predicate on the
// sorted sublist.  The sublist's own Step-3 samples (the items at ranks (k+1) w - 1, w = L/s)
// narrow it first: if c of them are <= g_j, then c w <= r_ij <= (c+1) w - 1 (a bisection over
// the s samples in LDS, one thread per j).  Then, for w <= 128, each wave counts inside the
// chunks of kRankBatch global samples at a time: all 64 lanes read one chunk's items with
// coalesced loads and a ballot counts those <= g_j, the loads of the whole batch in flight
// together (chunks shared by neighbouring samples come from cache).  Larger chunks are
// bisected in global memory, one probe per step.  Pads (x >= count) are key-max items.
constexpr uint32_t kRankBatch = 8;

// The chunk counts of k_rank for chunks of at most 64 NQ items: each wave takes kRankBatch
// global samples at a time (their chunks are wave-uniform), loads all their chunks, then counts.
template <class K, bool V, int NQ>
__device__ __forceinline__ void rank_chunks(const K *keys, const typename Tr<K, V>::SC *S,
                                            uint32_t m, const uint32_t *chunk, uint32_t *rk,
                                            uint32_t s, uint32_t w, uint32_t base,
                                            uint32_t count, uint32_t p0) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    const uint32_t lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t j0 = wv * kRankBatch; j0 < s; j0 += nwv * kRankBatch) {
        K v[kRankBatch][NQ];
        uint32_t cc[kRankBatch];  // wave-uniform chunk of each global sample of the batch
        SC gg[kRankBatch];        // and the global samples, loaded together with the chunks
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            cc[u] = j0 + u < s ? __builtin_amdgcn_readfirstlane(chunk[j0 + u]) : s;
            gg[u] = cc[u] < s ? S[(size_t)(j0 + u + 1) * m - 1] : SC{};
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t c = cc[u];
#pragma unroll
            for (uint32_t q = 0; q < NQ; ++q) {
                const uint32_t y = q * 64 + lane, x = c * w + y;  // item of the sublist
                v[u][q] = (c < s && y < w && x < count) ? keys[base + x] : KeyMax<K>::v;
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t j = j0 + u, c = cc[u];
            if (c >= s) continue;
            const SC g = gg[u];
            uint32_t le = 0;
#pragma unroll
            for (uint32_t q = 0; q < NQ; ++q) {
                const uint32_t y = q * 64 + lane;
                const bool in = y < w && !lt(g, R::samp(v[u][q], p0 + c * w + y));
                le += (uint32_t)__popcll(__ballot(in));
            }
            if (lane == 0) rk[j + 1] = c * w + le;
        }
    }
}

template <class K, bool V>
__global__ __launch_bounds__(256) void k_rank(const K *keys, const void *sorted_samples,
                                              const void *tile_samples, uint32_t *counts,
                                              SegView sv, uint32_t L, uint32_t s,
                                              uint32_t random) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    __shared__ uint32_t rk[1025], chunk[1024];
    __shared__ SC ts[1024];
    TileLoc loc;
    if (!locate_tile(sv, L, blockIdx.x, loc)) return;
    const uint32_t base = loc.seg_begin + loc.i * L;
    const uint32_t count = min(L, loc.seg_size - loc.i * L);
    const SC *S = (const SC *)sorted_samples + (size_t)loc.tile0 * s;
    const SC *T = (const SC *)tile_samples + (size_t)(loc.tile0 + loc.i) * s;
    for (uint32_t k = threadIdx.x; k < s; k += blockDim.x) ts[k] = T[k];
    __syncthreads();
    const uint32_t p0 = loc.i * L;
    const uint32_t w = L / s;
    if (random) {
        // Randomized samples (sorted run, at arbitrary positions): if c of them are <= g_j, the
        // rank lies after the position of sample c - 1 and at or before that of sample c, and is
        // bisected there in global memory.  +infinity closes the last bucket: r_is = L.
        for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
            if (j + 1 == s) {
                rk[s] = L;
                continue;
            }
            const SC g = S[(size_t)(j + 1) * loc.m - 1];
            uint32_t lo = 0, hi = s;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (!lt(g, ts[mid])) lo = mid + 1; else hi = mid;
            }
            uint32_t a = lo ? samp_pos(ts[lo - 1]) - p0 + 1 : 0u;
            uint32_t b = lo < s ? samp_pos(ts[lo]) - p0 : L;
            while (a < b) {
                const uint32_t x = (a + b) >> 1;
                const K kx = x < count ? keys[base + x] : KeyMax<K>::v;
                if (!lt(g, R::samp(kx, p0 + x))) a = x + 1; else b = x;
            }
            rk[j + 1] = a;
        }
        if (threadIdx.x == 0) rk[0] = 0;
        __syncthreads();
        uint32_t *row = counts + (size_t)(loc.tile0 + loc.i) * s;
        for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) row[j] = rk[j + 1] - rk[j];
        return;
    }
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        const SC g = S[(size_t)(j + 1) * loc.m - 1];
        uint32_t lo = 0, hi = s;  // c = #{k : sample_k <= g}
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (!lt(g, ts[mid])) lo = mid + 1; else hi = mid;
        }
        chunk[j] = lo;
        if (lo == s) rk[j + 1] = L;  // above every sample: above every item
    }
    if (threadIdx.x == 0) rk[0] = 0;
    __syncthreads();
    if (w <= 64) {
        rank_chunks<K, V, 1>(keys, S, loc.m, chunk, rk, s, w, base, count, p0);
    } else if (w <= 128) {
        rank_chunks<K, V, 2>(keys, S, loc.m, chunk, rk, s, w, base, count, p0);
    } else {
        for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
            const uint32_t c = chunk[j];
            if (c == s) continue;
            const SC g = S[(size_t)(j + 1) * loc.m - 1];
            uint32_t a = c * w, b = (c + 1) * w - 1;
            while (a < b) {
                const uint32_t x = (a + b) >> 1;
                const K kx = x < count ? keys[base + x] : KeyMax<K>::v;
                if (!lt(g, R::samp(kx, p0 + x))) a = x + 1; else b = x;
            }
            rk[j + 1] = a;
        }
    }
    __syncthreads();
    uint32_t *row = counts + (size_t)(loc.tile0 + loc.i) * s;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) row[j] = rk[j + 1] - rk[j];
}

// ------------------------------------------------------------------------------ Step 7

// Exclusive scan of v[0, n) in LDS (any n) by the first wave; returns the total.  Every
// thread of the block must call it.
__device__ uint32_t lds_scan(uint32_t *v, uint32_t n) {
    __shared__ uint32_t total;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        uint32_t carry = 0;
        for (uint32_t b = 0; b < n; b += 64) {
            const uint32_t j = b + lane;
            const uint32_t x = j < n ? v[j] : 0u;
            uint32_t inc = x;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d, 64);
                if (lane >= (uint32_t)d) inc += y;
            }
            if (j < n) v[j] = carry + inc - x;
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) total = carry;
    }
    __syncthreads();
    return total;
}

// Size classes of the final buckets: the scan kernels append every non-empty bucket to the
// work list of the smallest class that holds it, and one kernel per class (sized for that
// capacity) sorts the buckets on its list.
constexpr int kMaxClasses = 8;
struct Classes {
    uint32_t n;                  // 0: buckets feed another level instead
    uint32_t cap[kMaxClasses];   // ascending capacities (items)
    uint32_t *count;             // n counters, zeroed by k_init
    uint32_t *list;              // n lists of `stride` bucket indices
    uint32_t stride;
};

// Bucket table of one segment: {begin, real size, first piece, pieces}.  Pieces of bucket j are
// the m pieces A_1j..A_mj, stored bucket-major from `piece0 + j*m`.  Pads are the largest items,
// so after Step 8 they fill exactly [seg_size, n') of the segment; a bucket's real size is its
// overlap with [0, seg_size) (several trailing buckets may hold pads when the last sublist is
// mostly padding).  When asked, also the tile map of the next level: ceil(size / L_next)
// tiles per bucket, exclusive prefix, s + 1 entries.  `bucket0` is the global index of the
// segment's first bucket (for the class work lists).  A bucket of more than `limit` real items
// (randomized samples only; Algorithm 1's bound keeps every bucket within it) gets no tiles
// and no class: it is appended to `ovf_list` (count in *ovf_count) for a further run.
__device__ void emit_buckets(const uint32_t *colsum, const uint32_t *colbase, uint32_t s,
                             uint32_t seg_begin, uint32_t seg_size, uint32_t piece0, uint32_t m,
                             uint4 *buckets, uint32_t *tile_off_next, uint32_t L_next,
                             uint32_t *tmp, const Classes &cls, uint32_t bucket0,
                             uint32_t limit = 0xFFFFFFFFu, uint32_t *ovf_count = nullptr,
                             uint32_t *ovf_list = nullptr) {
    __shared__ uint32_t ccount[kMaxClasses], cbase[kMaxClasses];
    if (threadIdx.x < (uint32_t)kMaxClasses) ccount[threadIdx.x] = 0;
    __syncthreads();
    // class of each bucket and its slot among this workgroup's buckets of that class
    uint32_t mycls[4], myslot[4];
    for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t j = threadIdx.x + r * blockDim.x;
        mycls[r] = kMaxClasses;
        if (j >= s) continue;
        const uint32_t b = colbase[j];
        const uint32_t size = b >= seg_size ? 0u : min(colsum[j], seg_size - b);
        buckets[j] = make_uint4(seg_begin + b, size, piece0 + j * m, m);
        const bool over = size > limit && ovf_list;
        if (over) ovf_list[atomicAdd(ovf_count, 1u)] = bucket0 + j;  // at most s entries
        if (tile_off_next) tmp[j] = over ? 0u : (size + L_next - 1) / L_next;
        if (cls.n && size && !over) {
            uint32_t c = 0;
            while (c + 1 < cls.n && cls.cap[c] < size) ++c;
            mycls[r] = c;
            myslot[r] = atomicAdd(&ccount[c], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < cls.n && ccount[threadIdx.x])
        cbase[threadIdx.x] = atomicAdd(&cls.count[threadIdx.x], ccount[threadIdx.x]);
    __syncthreads();
    for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t j = threadIdx.x + r * blockDim.x;
        if (mycls[r] == (uint32_t)kMaxClasses) continue;
        const uint32_t at = cbase[mycls[r]] + myslot[r];
        if (at < cls.stride) cls.list[(size_t)mycls[r] * cls.stride + at] = bucket0 + j;
    }
    if (tile_off_next) {
        const uint32_t tot = lds_scan(tmp, s);
        for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) tile_off_next[j] = tmp[j];
        if (threadIdx.x == 0) tile_off_next[s] = tot;
    }
}

constexpr uint32_t kScanLds = 8192;  // entries of one row-block buffer

// For rows [r0, r1) of one segment (first row tile0, m rows, s columns) writes l_ij both
// row-major (`offs`) and bucket-major (`pdst`, entry tile0*s + j*m + i), and the source
// position of piece A_ij, seg_begin + i*L + sum_{j'<j} a_ij' (`psrc`, bucket-major).
// colstart[j] (LDS) holds l_{r0,j} on entry and is advanced.  C, Lm: LDS, kScanLds entries.
__device__ void scan_rows(const uint32_t *counts, uint32_t *offs, uint32_t *pdst, uint32_t *psrc,
                          uint32_t tile0, uint32_t m, uint32_t r0, uint32_t r1, uint32_t s,
                          uint32_t seg_begin, uint32_t L, uint32_t *colstart, uint32_t *C,
                          uint32_t *Lm) {
    const uint32_t tid = threadIdx.x, bd = blockDim.x;
    const uint32_t SB = kScanLds / s;
    const size_t pbase = (size_t)tile0 * s;
    for (uint32_t rb = r0; rb < r1; rb += SB) {
        const uint32_t nrow = min(SB, r1 - rb);
        const size_t rowq = (size_t)(tile0 + rb) * s;
        for (uint32_t q = tid; q < nrow * s; q += bd) C[q] = counts[rowq + q];
        __syncthreads();
        for (uint32_t j = tid; j < s; j += bd) {  // column prefix: l_ij
            uint32_t run = colstart[j];
            for (uint32_t r = 0; r < nrow; ++r) {
                Lm[r * s + j] = run;
                run += C[r * s + j];
            }
            colstart[j] = run;
        }
        __syncthreads();
        {  // row prefix in place: C becomes the start rank of each piece in its sublist
            const uint32_t lane = tid & 63, w = tid >> 6, nw = bd >> 6;
            for (uint32_t r = w; r < nrow; r += nw) {
                uint32_t carry = 0;
                for (uint32_t b = 0; b < s; b += 64) {
                    const uint32_t j = b + lane;
                    const uint32_t x = j < s ? C[r * s + j] : 0u;
                    uint32_t inc = x;
#pragma unroll
                    for (int d = 1; d < 64; d <<= 1) {
                        const uint32_t y = __shfl_up(inc, d, 64);
                        if (lane >= (uint32_t)d) inc += y;
                    }
                    if (j < s) C[r * s + j] = carry + inc - x;
                    carry += __shfl(inc, 63, 64);
                }
            }
        }
        __syncthreads();
        for (uint32_t q = tid; q < nrow * s; q += bd) offs[rowq + q] = Lm[q];
        for (uint32_t q = tid; q < nrow * s; q += bd) {
            const uint32_t r = q % nrow, j = q / nrow;
            const size_t e = pbase + (size_t)j * m + rb + r;
            pdst[e] = Lm[r * s + j];
            psrc[e] = seg_begin + (rb + r) * L + C[r * s + j];
        }
        __syncthreads();
    }
}

// Step 7 for many segments, one workgroup each (second level): column sums, their exclusive
// scan (bucket starts), the bucket table, then every l_ij and piece source.
__global__ __launch_bounds__(256) void k_scan_seg(const uint32_t *counts, uint32_t *offs,
                                                  uint32_t *pdst, uint32_t *psrc, SegView sv,
                                                  uint32_t L, uint32_t s, uint4 *buckets,
                                                  Classes cls) {
    __shared__ uint32_t colsum[1024], colbase[1024], C[kScanLds], Lm[kScanLds];
    const uint32_t g = blockIdx.x;
    if (sv.tile_off[g + 1] > sv.max_tiles) return;
    const uint32_t tile0 = sv.tile_off[g];
    const uint32_t m = sv.tile_off[g + 1] - tile0;
    if (m == 0) return;  // no tiles: no buckets (they are never on a work list)
    const uint32_t seg_begin = sv.seg[g].x, seg_size = sv.seg[g].y;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t sum = 0;
#pragma unroll 8
        for (uint32_t i = 0; i < m; ++i) sum += counts[(size_t)(tile0 + i) * s + j];
        colsum[j] = sum;
        colbase[j] = sum;
    }
    lds_scan(colbase, s);
    emit_buckets(colsum, colbase, s, seg_begin, seg_size, tile0 * s, m, buckets + (size_t)g * s,
                 nullptr, 0u, nullptr, cls, g * s);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) colsum[j] = seg_begin + colbase[j];
    __syncthreads();
    scan_rows(counts, offs, pdst, psrc, tile0, m, 0, m, s, seg_begin, L, colsum, C, Lm);
}

// Step 7 for one segment [0, n) with many sublists, in three kernels: (a) column sums of each
// block of RB rows, (b) one workgroup scans them per column and across columns, (c) every row
// block writes its l_ij and piece sources.
__global__ __launch_bounds__(256) void k_scan_partial(const uint32_t *counts, uint32_t *partial,
                                                      uint32_t m, uint32_t s, uint32_t RB) {
    const uint32_t i0 = blockIdx.x * RB, i1 = min(m, i0 + RB);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t sum = 0;
#pragma unroll 8
        for (uint32_t i = i0; i < i1; ++i) sum += counts[(size_t)i * s + j];
        partial[(size_t)blockIdx.x * s + j] = sum;
    }
}

// (b): groups of s threads each take a contiguous share of the row blocks of every column:
// column sums per share, their prefix across shares, then each share's row-block prefixes
// written back into `partial` (column-relative; k_scan_apply adds the bucket's start).
__global__ __launch_bounds__(1024) void k_scan_mid(uint32_t *partial, uint32_t nrb, uint32_t m,
                                                   uint32_t s, uint32_t n, uint4 *buckets,
                                                   uint32_t *tile_off_next, uint32_t L_next,
                                                   Classes cls, uint32_t limit,
                                                   uint32_t *ovf_count, uint32_t *ovf_list) {
    __shared__ uint32_t colsum[1024], colbase[1024], tmp[1024];
    const uint32_t ng = blockDim.x / s;  // s divides blockDim (both powers of two, s <= 1024)
    const uint32_t grp = threadIdx.x / s, j = threadIdx.x % s;
    const uint32_t per = (nrb + ng - 1) / ng;
    const uint32_t b0 = min(nrb, grp * per), b1 = min(nrb, b0 + per);
    uint32_t own = 0;
#pragma unroll 8
    for (uint32_t b = b0; b < b1; ++b) own += partial[(size_t)b * s + j];
    tmp[grp * s + j] = own;
    __syncthreads();
    uint32_t run = 0;
    for (uint32_t q = 0; q < grp; ++q) run += tmp[q * s + j];
    if (grp == ng - 1) {
        colsum[j] = run + own;
        colbase[j] = run + own;
    }
#pragma unroll 8
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t x = partial[(size_t)b * s + j];
        partial[(size_t)b * s + j] = run;
        run += x;
    }
    lds_scan(colbase, s);  // (starts with a barrier: tmp is free again after it)
    emit_buckets(colsum, colbase, s, 0u, n, 0u, m, buckets, tile_off_next, L_next, tmp, cls, 0u,
                 limit, ovf_count, ovf_list);
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *counts, const uint32_t *partial,
                                                    const uint4 *buckets, uint32_t *offs,
                                                    uint32_t *pdst, uint32_t *psrc, uint32_t m,
                                                    uint32_t s, uint32_t RB, uint32_t L) {
    __shared__ uint32_t colstart[1024], C[kScanLds], Lm[kScanLds];
    const uint32_t i0 = blockIdx.x * RB, i1 = min(m, i0 + RB);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x)
        colstart[j] = buckets[j].x + partial[(size_t)blockIdx.x * s + j];
    __syncthreads();
    scan_rows(counts, offs, pdst, psrc, 0u, m, i0, i1, s, 0u, L, colstart, C, Lm);
}

// ------------------------------------------------------------------------------ Steps 8+9

struct GatherArgs {
    const void *src_keys;    // sorted sublists of the last level
    void *dst_keys;          // output (must not alias src)
    const uint32_t *src_vals;
    uint32_t *dst_vals;
    const uint4 *buckets;    // {begin, size, first piece, pieces}
    const uint32_t *pdst;    // bucket-major l_ij
    const uint32_t *psrc;    // bucket-major source position of A_ij
    uint32_t *count;         // per class: buckets on its list; the class's work-queue
                             // counter sits 2 * kMaxClasses entries further on
    const uint32_t *list;    // per class: bucket indices
    uint32_t stride;
    uint32_t n_total;
    uint32_t *status;
};

constexpr uint32_t kMaxPieces = 256;

// Items per thread of the merge-sort bucket kernels: 16 (8 for 16-byte elements and for
// key/value sorts, whose kernels also ask for at least four waves per SIMD), 20 for the 10K
// class of 32-bit keys (its buckets then take as many merge passes as the 8K class), raised so
// that CAP / E <= 1024 threads.
template <class K, bool V, int CAP> struct GatherE {
    static constexpr bool keys32 = !V && sizeof(K) == 4;
    static constexpr int base = sizeof(typename Tr<K, V>::T) >= 16 ? 8
                                : V                                 ? 8
                                : keys32 && CAP == 10240            ? 20
                                                                    : 16;
    static constexpr int E = CAP / base > 1024 ? (CAP / 1024 <= 16 ? 16 : 32) : base;
    static constexpr int wpe = V ? 4 : 1;
    static_assert(CAP % E == 0 && CAP / E <= 1024 && (CAP / E) % 64 == 0, "bucket class shape");
};


// Steps 8 and 9 fused: the pieces of a bucket are gathered into LDS, each wave streaming its
// share of the bucket with every lane following the piece its item is in (with their bucket
// positions as tie-breaks for key/value sorts), padded with key-max
// items to a multiple of E, and sorted with the block merge sort.  One workgroup of CAP / E
// threads per bucket of at most CAP items; persistent over the class's work list, taking
// buckets from a queue counter (zeroed by k_init) so that workgroups that are not resident at
// first, and ones that drew small buckets, share the work evenly.
template <class K, bool V, int CAP, bool XOUT, bool XIN = false>
__global__ __launch_bounds__((CAP / GatherE<K, V, CAP>::E), (GatherE<K, V, CAP>::wpe))
    void k_gather_bsort(GatherArgs a, uint32_t cls) {
    using R = Tr<K, V>;
    using T = typename R::T;
    constexpr int E = GatherE<K, V, CAP>::E;
    constexpr uint32_t BD = CAP / E;
    __shared__ T lds[lds_elems<T>(CAP) + 1];
    __shared__ uint32_t bnd[kMaxPieces + 1], ps[kMaxPieces];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, w = tid >> 6, nw = BD >> 6;
    __shared__ uint32_t slot[2];
    const uint32_t nwork = min(a.count[cls], a.stride);
    const uint32_t *list = a.list + (size_t)cls * a.stride;
    uint32_t *queue = a.count + 2 * kMaxClasses + cls;
    const K *src = (const K *)a.src_keys;
    K *dst = (K *)a.dst_keys;
    if (blockIdx.x >= nwork) return;  // more workgroups than buckets: nothing to take
    if (tid == 0) slot[0] = atomicAdd(queue, 1u);
    __syncthreads();
    for (uint32_t k = 0;; k ^= 1) {
        // slot[k] was written before the previous barrier; slot[k ^ 1] was last read at the
        // top of the previous iteration, before its barriers
        // uniform: keeps the bucket's description in scalar registers
        const uint32_t item = __builtin_amdgcn_readfirstlane(slot[k]);
        if (item >= nwork) break;
        const uint4 b = a.buckets[list[item]];
        const uint32_t begin = b.x, total = b.y, pbase = b.z, np = b.w;
        if (total == 0 || total > CAP || np > kMaxPieces || np == 0 ||
            (uint64_t)begin + total > a.n_total) {
            if (tid == 0) {
                atomicOr(a.status, 8u);
                slot[k ^ 1] = atomicAdd(queue, 1u);
            }
            __syncthreads();
            continue;
        }
        __syncthreads();
        for (uint32_t i = tid; i < np; i += BD) {
            bnd[i] = min(a.pdst[pbase + i] - begin, total);
            ps[i] = a.psrc[pbase + i];
        }
        if (tid == 0) bnd[np] = total;
        __syncthreads();
        // padded to whole runs of the block sort's first pass (256 items where it merges in
        // registers first, else E)
        constexpr uint32_t PR = (sizeof(T) == 4 && E == 16) ? 256 : E;
        const uint32_t P = (total + PR - 1) / PR * PR;
        const uint32_t span = ((P + nw - 1) / nw + 63) & ~63u;
        const uint32_t x_begin = w * span, x_end = min(P, x_begin + span);
        if (x_begin < x_end) {
            uint32_t p = 0;
            {
                uint32_t lo = 0, hi = np - 1;
                const uint32_t xs = min(x_begin + lane, total - 1);
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (bnd[mid] <= xs) lo = mid; else hi = mid - 1;
                }
                p = lo;
            }
            for (uint32_t row = x_begin; row < x_end; row += 4 * 64) {
                K v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t xu = row + 64 * u + lane;
                    if (xu < total) {
                        while (xu >= bnd[p + 1]) ++p;
                        v[u] = src[ps[p] + (xu - bnd[p])];
                        if (XIN) v[u] = (K)f32_in((uint32_t)v[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t xu = row + 64 * u + lane;
                    if (xu < x_end) lds[pidx<T>(xu)] = xu < total ? R::make(v[u], xu) : R::pad(xu);
                }
            }
        }
        __syncthreads();
        block_sort<T, E, V>(lds, P);  // key/value elements carry their gathered position
        uint32_t nxt = 0;  // the next bucket, requested while this one is written out
        if (tid == 0) nxt = atomicAdd(queue, 1u);

        // two at a time: unrolled whole, the loads and store addresses in flight would set
        // the kernel's register count (and so its occupancy)
#pragma unroll 2
        for (int q = 0; q < E; ++q) {
            const uint32_t x = tid + q * BD;
            if (x < total) {
                K kk = R::key(lds[pidx<T>(x)]);
                if (XOUT) kk = (K)f32_out((uint32_t)kk);
                dst[begin + x] = kk;
            }
        }
        if constexpr (V) {
            __syncthreads();
            for (uint32_t i = w; i < np; i += nw) {
                const uint32_t d0 = bnd[i], len = bnd[i + 1] - d0, s0 = ps[i];
                for (uint32_t q = lane; q < len; q += 64)
                    put_val<T>(lds, d0 + q, a.src_vals[s0 + q]);
            }
            __syncthreads();
#pragma unroll 2
            for (int q = 0; q < E; ++q) {
                const uint32_t x = tid + q * BD;
                if (x < total) a.dst_vals[begin + x] = val_of_sorted<T>(lds, x);
            }
        }
        if (tid == 0) slot[k ^ 1] = nxt;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------ misc

// The workspace's first 256 bytes: [0] status flags, [1, 1 + kMaxClasses) the final buckets'
// class counters, [1 + kMaxClasses, 1 + 2 kMaxClasses) those of a segmented sort's one-piece
// buckets, 2 kMaxClasses entries after each counter its class's work-queue counter, and at
// kOverflowWord the count of a randomized call's buckets routed to a further run.
static_assert(kOverflowWord > 4u * kMaxClasses && kOverflowWord < 64u, "status page layout");
__global__ void k_init(uint32_t *status) {
    if (threadIdx.x < 64u && blockIdx.x == 0) status[threadIdx.x] = 0;
}

// Long-segment classes of a segmented sort, as the set-up kernel sees them.
struct SegClassArgs {
    uint32_t n;                           // classes
    uint32_t hi[kMaxSegClasses];          // class c: lengths in (hi[c-1], hi[c]]
    uint32_t L[kMaxSegClasses];
    uint32_t gmax[kMaxSegClasses];        // room in the class's tables
    uint4 *tab[kMaxSegClasses];           // {begin, size, 0, 0} per segment of the class
    uint32_t *tile_off[kMaxSegClasses];   // gmax + 1 entries
};

// Segmented sort set-up, one workgroup.  From the caller's CSR offsets (S + 1 uint64):
//  * every segment that fits one workgroup (0 < size <= small_cap) becomes a one-piece bucket
//    {begin, size, g, 1} on the work list of its size class;
//  * every longer one goes, in input order, to the compact table of its length class, with the
//    class's tile map (ceil(size / L) tiles each, exclusive prefix); unused entries up to the
//    class's room are empty segments with no tiles.
// Offsets that decrease or pass n would let segments overlap or leave the array: then no
// segment is sorted and status bit 16 is set.  A segment longer than max_seg is left as it is
// and sets bit 32.
__global__ __launch_bounds__(1024) void k_seg_prepare(const uint64_t *off, uint32_t S, uint32_t n,
                                                      uint32_t max_seg, uint32_t small_cap,
                                                      SegClassArgs ca, uint4 *small_b,
                                                      uint32_t *spiece, Classes cls,
                                                      uint32_t *status) {
    __shared__ uint32_t wsum[17];
    __shared__ uint32_t carry_t[kMaxSegClasses], carry_g[kMaxSegClasses], malformed;
    if (threadIdx.x < (uint32_t)kMaxSegClasses) carry_t[threadIdx.x] = carry_g[threadIdx.x] = 0;
    if (threadIdx.x == 0) malformed = off[S] > n ? 1u : 0u;
    __syncthreads();
    for (uint32_t g = threadIdx.x; g < S; g += blockDim.x)
        if (off[g + 1] < off[g]) malformed = 1u;
    __syncthreads();
    const bool skip_all = malformed != 0;
    if (skip_all && threadIdx.x == 0) atomicOr(status, 16u);
    for (uint32_t b0 = 0; b0 < S; b0 += blockDim.x) {
        const uint32_t g = b0 + threadIdx.x;
        uint32_t begin = 0, size = 0;
        if (g < S && !skip_all) {
            const uint64_t lo = off[g], hi = off[g + 1];
            if (hi - lo > max_seg) {
                atomicOr(status, 32u);
            } else {
                begin = (uint32_t)lo;
                size = (uint32_t)(hi - lo);
            }
            if (size > 0 && size <= small_cap) {
                small_b[g] = make_uint4(begin, size, g, 1u);
                spiece[g] = begin;
                uint32_t c = 0;
                while (c + 1 < cls.n && cls.cap[c] < size) ++c;
                const uint32_t at = atomicAdd(&cls.count[c], 1u);
                if (at < cls.stride) cls.list[(size_t)c * cls.stride + at] = g;
            }
        }
        uint32_t mine = kMaxSegClasses;  // length class of a long segment
        if (size > small_cap) {
            mine = 0;
            while (mine + 1 < ca.n && size > ca.hi[mine]) ++mine;
        }
        for (uint32_t c = 0; c < ca.n; ++c) {
            bool in = mine == c;
            uint32_t tot_t, tot_g;
            const uint32_t ex_g = block_excl_scan(in ? 1u : 0u, wsum, tot_g);
            const uint32_t idx = carry_g[c] + ex_g;
            if (in && idx >= ca.gmax[c]) {  // cannot happen for disjoint segments inside [0, n)
                atomicOr(status, 16u);
                in = false;
            }
            const uint32_t ex_t =
                block_excl_scan(in ? (size + ca.L[c] - 1) / ca.L[c] : 0u, wsum, tot_t);
            if (in) {
                ca.tab[c][idx] = make_uint4(begin, size, 0u, 0u);
                ca.tile_off[c][idx] = carry_t[c] + ex_t;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                carry_t[c] += tot_t;
                carry_g[c] = min(carry_g[c] + tot_g, ca.gmax[c]);
            }
            __syncthreads();
        }
    }
    for (uint32_t c = 0; c < ca.n; ++c)
        for (uint32_t i = carry_g[c] + threadIdx.x; i <= ca.gmax[c]; i += blockDim.x) {
            ca.tile_off[c][i] = carry_t[c];
            if (i < ca.gmax[c]) ca.tab[c][i] = make_uint4(0u, 0u, 0u, 0u);
        }
}

// Step 8 as the paper states it, for the level-1 buckets of a randomized call that are routed
// to a further run: every piece A_ij of every listed bucket is copied from the sorted sublists
// (src) to its place l_ij in dst, clipped to the bucket's real items (pads, the largest items,
// sit at the end of the last piece and are dropped).  One wave per piece, grid-stride over
// (listed bucket, piece); xout applies the f32 order map's inverse on the way.
template <class K>
__global__ __launch_bounds__(256) void k_reloc_listed(const K *src, K *dst, const uint32_t *src_vals,
                                                      uint32_t *dst_vals, const uint4 *buckets,
                                                      const uint32_t *pdst, const uint32_t *psrc,
                                                      const uint32_t *ovf_count,
                                                      const uint32_t *ovf_list, uint32_t s,
                                                      uint32_t m, uint32_t n_total,
                                                      uint32_t xout) {
    const uint32_t nb = min(*ovf_count, s);
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nwave = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t q = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
         q < (uint64_t)nb * m; q += nwave) {
        const uint32_t bi = (uint32_t)(q / m), p = (uint32_t)(q % m);
        const uint4 b = buckets[ovf_list[bi]];
        if (p >= b.w) continue;
        const uint32_t end = min(b.x + b.y, n_total);
        const uint32_t d0 = min(pdst[b.z + p], end);
        const uint32_t d1 = min(p + 1 < b.w ? pdst[b.z + p + 1] : end, end);
        const uint32_t s0 = psrc[b.z + p];
        for (uint32_t x = lane; d0 + x < d1 && s0 + x < n_total; x += 64) {
            K k = src[s0 + x];
            if (xout) k = (K)f32_out((uint32_t)k);
            dst[d0 + x] = k;
            if (dst_vals) dst_vals[d0 + x] = src_vals[s0 + x];
        }
    }
}

// Copies the listed buckets' ranges [begin, begin + size) from src to dst (randomized calls of
// two levels: their relocated items move from the workspace copy back into the keys).
template <class K>
__global__ __launch_bounds__(256) void k_copy_listed(const K *src, K *dst, const uint32_t *src_vals,
                                                     uint32_t *dst_vals, const uint4 *buckets,
                                                     const uint32_t *ovf_count,
                                                     const uint32_t *ovf_list, uint32_t s,
                                                     uint32_t n_total, uint32_t xout) {
    const uint32_t nb = min(*ovf_count, s);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t bi = 0; bi < nb; ++bi) {
        const uint4 b = buckets[ovf_list[bi]];
        const uint32_t end = min(b.x + b.y, n_total);
        for (uint32_t x = b.x + blockIdx.x * blockDim.x + threadIdx.x; x < end; x += stride) {
            K k = src[x];
            if (xout) k = (K)f32_out((uint32_t)k);
            dst[x] = k;
            if (dst_vals) dst_vals[x] = src_vals[x];
        }
    }
}

// Clears the work-list counters of the final buckets and their queue counters (between the
// classes of a segmented sort).
__global__ void k_clear_counters(uint32_t *count, uint32_t n) {
    if (threadIdx.x < n) {
        count[threadIdx.x] = 0;
        count[threadIdx.x + 2 * kMaxClasses] = 0;
    }
}

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
                      q.L, q.s, 0u);
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
                       nullptr, g.seed, rnd};
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
                  (const void *)sorted, (const void *)samp, counts, sv1, g.L1, g.s1, rnd);
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
            TileArgs a{keys, wkeys, d_vals, wvals, sv2, g.L2, g.s2, samp2, status, pdst, psrc};
            DS_LAUNCH("s8_l2_s123_gather_sort",
                      (k_tile<K, V, TE, TCAP, MODE_SAMPLE, false, false, true>),
                      dim3(g.tiles2max), dim3(g.L2 / TE), a);
        }
        rc = sort_samples(samp2, sorted2, nullptr, sv2, g.L2, g.s2, g.s1, 0, status, st, false, 0,
                          tm, "l2_s4_sample_sort", "l2_s4_sample_merge");
        if (rc) return rc;
        DS_LAUNCH("l2_s56_rank", (k_rank<K, V>), dim3(g.tiles2max), dim3(256), (const K *)wkeys,
                  (const void *)sorted2, (const void *)samp2, counts2, sv2, g.L2, g.s2, 0u);
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
