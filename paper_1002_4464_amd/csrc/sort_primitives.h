// Device building blocks of the sort kernels (gfx950, wave64): element types and their
// order, the f32 totalOrder map, segment and tile addressing, the block sort (register
// network, in-register DPP / ds_swizzle merges, LDS merge-path passes) and wave and block
// scans.  Included once, by kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Merges of 32-bit keys (no positions) on a bitonic layout: in every run pair the first run
// A is stored ascending and the second run B descending, so that reading past the end of
// either run reads the other run's largest items instead of unrelated ones.  A thread that
// has used up A then sees B's maximum: it takes B's items until the one it reads from B's
// end equals the B item it holds, and then every item left is that maximum, so the values it
// outputs are right whichever side it takes them from.  A thread that has used up B sees A's
// maximum and takes A, as it must.  So the serial merge needs no bounds tests.  The pointers of
// one thread never cross, because it outputs no more items than the pair has left, so every
// read stays in [base, base + na + nb] (the element one past the pair is read, unused, when a
// thread's outputs end at the pair's end).

// Merge-path split of the first `diag` outputs of A = lds[base, base + na) (ascending) and B
// (nb items, descending from base + na + nb - 1): the largest a whose A[a - 1] does not follow
// B[diag - a], by the same clamped halving steps as merge_split.
__device__ __forceinline__ uint32_t merge_split_bit(const uint32_t *lds, uint32_t base,
                                                    uint32_t na, uint32_t nb, uint32_t diag,
                                                    uint32_t top) {
    const uint32_t lo = diag > nb ? diag - nb : 0, hi = min(diag, na);
    uint32_t pos = lo;
    if (lo < hi) {
        const uint32_t am1 = base - 1, br = base + na + nb - 1 - diag;  // A[q-1], B[diag-q]
        for (uint32_t step = top; step; step >>= 1) {
            const uint32_t q = min(pos + step, hi);
            const uint32_t av = lds_at<uint32_t>(lds, am1 + q);
            const uint32_t bv = lds_at<uint32_t>(lds, br + q);
            pos = bv < av ? pos : q;
        }
    }
    return pos;
}

// Serial merge of E outputs on the bitonic layout: pa walks A upwards, pb walks B downwards
// (B's next item is at pb); A wins ties.  pa and pb are left at the next unmerged items.
template <int E>
__device__ __forceinline__ void serial_merge_bit(const uint32_t *lds, uint32_t &pa, uint32_t &pb,
                                                 uint32_t (&out)[E]) {
    uint32_t av = lds_at<uint32_t>(lds, pa);
    uint32_t bv = lds_at<uint32_t>(lds, pb);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t ta = bv >= av ? 1u : 0u;
        // keys alone: the output is the smaller head, whichever side it comes from; pinned
        // here (an empty asm) so that the compiler does not keep both heads of every step
        // alive until the stores
        out[k] = min(av, bv);
        asm volatile("" : "+v"(out[k]));
        pa += ta;
        pb = pb + ta - 1u;
        // both pointers as plain registers: left alone, the compiler re-derives them from
        // running sums of the take flags, one more compare and select per step
        asm("" : "+v"(pa), "+v"(pb));
        const uint32_t v = lds_at<uint32_t>(lds, ta ? pa : pb);
        av = ta ? v : av;
        bv = ta ? bv : v;
    }
}

// Stores E registers into the block lds[blk, blk + E) (blk a multiple of E; padded indexing),
// in order or reversed.  When E is a power of two within one padding period the block never
// straddles a pad, so each store is one immediate offset from a common address.  Otherwise
// every item's padded index is computed, walking the block upwards or downwards with one
// code path for both (two branches would both run in waves holding pairs of either parity).
template <class T, int E>
__device__ __forceinline__ void store_block(T *lds, uint32_t blk, bool rev, const T (&x)[E]) {
    if constexpr ((E & (E - 1)) == 0 && E <= (1 << PadShift<T>::v)) {
        blk &= ~(uint32_t)(E - 1);
        T *p = lds + pidx<T>(blk);
        if (rev) {
#pragma unroll
            for (int k = 0; k < E; ++k) p[E - 1 - k] = x[k];
        } else {
#pragma unroll
            for (int k = 0; k < E; ++k) p[k] = x[k];
        }
    } else {
        uint32_t i = rev ? blk + E - 1 : blk;
        uint32_t step = rev ? 0xFFFFFFFFu : 1u;
        asm volatile("" : "+v"(i), "+v"(step));
#pragma unroll
        for (int k = 0; k < E; ++k) {
            lds[pidx<T>(i)] = x[k];
            i += step;
        }
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
// Keys-only 32-bit sorts merge on the bitonic layout (see merge_split_bit), so their serial
// merges carry no bounds tests.
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
    const uint32_t Rs = R0 > E         ? R0
                        : dpp64   ? 64 * E
                        : dpp32   ? 32 * E
                        : dpp16   ? 16 * E
                        : dpp     ? 8 * E
                                  : E;
    // keys-only 32-bit merges run on the bitonic layout (odd runs stored descending)
    constexpr bool BIT = sizeof(T) == 4 && !COMP;
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
        const uint32_t run = t * E / Rs;  // P is a multiple of Rs: every run is full
        if (BIT && Rs < P) {
            const bool rev = run & 1;  // odd runs descending: block t goes to its mirror
            store_block<T, E>(lds, rev ? 2 * run * Rs + Rs - E - t * E : t * E, rev, x);
        } else {
#pragma unroll
            for (int k = 0; k < E; ++k) lds[pidx<T>(t * E + k)] = x[k];
        }
    }
    if constexpr (BIT) {
        const bool two = TWO && P % (2 * E) == 0;
        const uint32_t EB = two ? 2 * E : E;  // outputs per active thread
        const bool actb = t * EB < P;
        for (uint32_t R = Rs, pair = 2 * Rs / E, top = pow2_at_least(Rs); R < P;
             R <<= 1, pair <<= 1, top <<= 1) {
            __syncthreads();
            // a pair holds 2R items: pair threads of E outputs (pair / 2 of 2E outputs)
            const uint32_t tp = two ? pair / 2 : pair;
            const uint32_t base = (t & ~(tp - 1)) * EB;  // first item of the thread's run pair
            const uint32_t diag = t * EB - base;
            const uint32_t na = min(R, P - base);
            const uint32_t nb = min(R, P - base - na);
            T y[E];
            if (actb) {
                const uint32_t a = merge_split_bit(lds, base, na, nb, diag, top);
                uint32_t pa = base + a, pb = base + na + nb - 1 - (diag - a);
                serial_merge_bit<E>(lds, pa, pb, x);
                if (two) serial_merge_bit<E>(lds, pa, pb, y);
            }
            __syncthreads();
            if (actb) {
                // the merged run is the next pass's A (ascending) or B (descending); the last
                // pass leaves everything ascending
                const bool desc = 2 * R < P && (t & tp);  // odd pair: B of the next pass
                // na, nb, diag are multiples of E: output block q of the thread lands on an
                // E-aligned block, at its mirror image in the pair when descending
                const uint32_t mir = base + na + nb - E - diag;
                store_block<T, E>(lds, desc ? mir : base + diag, desc, x);
                if (two) store_block<T, E>(lds, desc ? mir - E : base + diag + E, desc, y);
            }
        }
        __syncthreads();
        return;
    }
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


}  // namespace
}  // namespace dsort
