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
//   k_relocate            Step 8: move each piece A_ij to l_ij.
//   k_tile<MODE_FINAL>    Step 9: sort each bucket B_j inside one workgroup.
// For inputs where one level would need too many samples, Step 9 runs Algorithm 1 again on
// every bucket (the buckets become the segments of a second level).
//
// Order: items compare under the total order (key, sublist i, sorted rank r); samples are the
// composites (key, i*L + r).  float32 keys are mapped to their IEEE totalOrder image on the
// first load and back on the last store, so every intermediate holds unsigned order keys.
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

// ------------------------------------------------------------------------------ segments

// A set of segments (independent sort problems) and their partition into tiles of L items.
// seg == nullptr means one segment [0, n_single).
struct SegView {
    const uint2 *seg;          // {begin, size} per segment
    const uint32_t *tile_off;  // G+1 entries: exclusive prefix of ceil(size/L) over segments
    uint32_t G;
    uint32_t n_single;
    uint32_t n_total;          // length of the keys array the segments index
    uint32_t max_tiles;        // capacity of the per-tile tables (tile_off views)
};

struct TileLoc {
    uint32_t g, i, seg_begin, seg_size, tile0, m;
};

__device__ __forceinline__ bool locate_tile(const SegView &sv, uint32_t L, uint32_t t,
                                            TileLoc &o) {
    if (!sv.tile_off) {
        const uint32_t m = (sv.n_single + L - 1) / L;
        if (t >= m) return false;
        o.g = 0; o.i = t; o.seg_begin = 0; o.seg_size = sv.n_single; o.tile0 = 0; o.m = m;
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
    const uint2 d = sv.seg[lo];
    o.seg_begin = d.x;
    o.seg_size = d.y;
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
    const T lo = sw ? b : a;
    const T hi = sw ? a : b;
    a = lo;
    b = hi;
}

// Batcher's odd-even merge sort network over E registers (E a power of two).
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

// Merge path: number of A items among the first `diag` outputs of the stable merge of
// A = lds[a0, a0+na) and B = lds[b0, b0+nb) (A wins ties).
template <class T>
__device__ __forceinline__ uint32_t merge_path(const T *lds, uint32_t a0, uint32_t na,
                                               uint32_t b0, uint32_t nb, uint32_t diag) {
    uint32_t lo = diag > nb ? diag - nb : 0;
    uint32_t hi = diag < na ? diag : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const T av = lds[pidx<T>(a0 + mid)];
        const T bv = lds[pidx<T>(b0 + diag - 1 - mid)];
        if (lt(bv, av)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Serial stable merge of E outputs starting at A index ai (< a_end) / B index bi (< b_end).
// `lim` is any valid LDS index used to keep speculative reads in bounds.
template <class T, int E>
__device__ __forceinline__ void serial_merge(const T *lds, uint32_t ai, uint32_t a_end,
                                             uint32_t bi, uint32_t b_end, uint32_t lim,
                                             T (&out)[E]) {
    T av = lds[pidx<T>(min(ai, lim))];
    T bv = lds[pidx<T>(min(bi, lim))];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const bool take_a = (bi >= b_end) || ((ai < a_end) && !lt(bv, av));
        out[k] = take_a ? av : bv;
        const uint32_t nxt = take_a ? ai + 1 : bi + 1;
        ai = take_a ? ai + 1 : ai;
        bi = take_a ? bi : bi + 1;
        const T v = lds[pidx<T>(min(nxt, lim))];
        av = take_a ? v : av;
        bv = take_a ? bv : v;
    }
}

// Sorts lds[0, P) in place (P a power of two, E <= P <= E * blockDim.x).  Thread t owns
// items [tE, tE+E): a register network sorts them, then log2(P/E) merge passes double the
// sorted run length.  All threads of the block must call it.
template <class T, int E> __device__ void block_sort(T *lds, uint32_t P) {
    const uint32_t t = threadIdx.x;
    const bool act = t * E < P;
    T x[E];
    if (act) {
#pragma unroll
        for (int k = 0; k < E; ++k) x[k] = lds[pidx<T>(t * E + k)];
        reg_sort<T, E>(x);
#pragma unroll
        for (int k = 0; k < E; ++k) lds[pidx<T>(t * E + k)] = x[k];
    }
    for (uint32_t R = E; R < P; R <<= 1) {
        __syncthreads();
        if (act) {
            const uint32_t start = t * E;
            const uint32_t base = start & ~(2 * R - 1);
            const uint32_t diag = start - base;
            const uint32_t a = merge_path<T>(lds, base, R, base + R, R, diag);
            serial_merge<T, E>(lds, base + a, base + R, base + R + diag - a, base + 2 * R,
                               base + 2 * R - 1, x);
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < E; ++k) lds[pidx<T>(t * E + k)] = x[k];
        }
    }
    __syncthreads();
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
};

// MODE_SAMPLE (Steps 1-3): one workgroup per sublist of L items; writes the sorted sublist in
// place and its s samples.  MODE_FINAL (Step 9): one workgroup per segment of at most CAP
// items, sorted from src into dst (which may alias).  XIN/XOUT apply the f32 order map.
template <class K, bool V, int E, int CAP, int MODE, bool XIN, bool XOUT>
__global__ __launch_bounds__(CAP / E) void k_tile(TileArgs a) {
    using R = Tr<K, V>;
    using T = typename R::T;
    __shared__ T lds[lds_elems<T>(CAP)];
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
        uint2 d = a.sv.seg ? a.sv.seg[blockIdx.x] : make_uint2(0u, a.sv.n_single);
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
    __syncthreads();
    block_sort<T, E>(lds, P);

    if (MODE == MODE_SAMPLE) {
        typename R::SC *smp = (typename R::SC *)a.samples;
        const uint32_t w = a.L / a.s;
        for (uint32_t k = tid; k < a.s; k += bd) {
            const uint32_t r = (k + 1) * w - 1;
            smp[(size_t)(loc.tile0 + loc.i) * a.s + k] = R::samp(R::key(lds[pidx<T>(r)]), loc.i * a.L + r);
        }
    }

    K *dst = (K *)a.dst_keys;
    uint32_t pos[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const uint32_t i = tid + q * bd;
        if (i < count) {
            const T e = lds[pidx<T>(i)];
            K k = R::key(e);
            if (XOUT) k = (K)f32_out((uint32_t)k);
            dst[begin + i] = k;
            pos[q] = R::lpos(e);
        }
    }
    if (V) {
        __syncthreads();
        uint32_t *lv = (uint32_t *)lds;
        for (uint32_t i = tid; i < count; i += bd) lv[i] = a.src_vals[begin + i];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * bd;
            if (i < count) a.dst_vals[begin + i] = lv[pos[q]];
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
    __shared__ SC lds[lds_elems<SC>(CAP)];
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
    block_sort<SC, E>(lds, P);
    for (uint32_t i = tid; i < count; i += blockDim.x) dst[begin + i] = lds[pidx<SC>(i)];
}

// One round of a global merge sort over sorted runs of length R (R a multiple of CAP):
// workgroup b writes outputs [b*CAP, (b+1)*CAP) of the merge of its run pair.
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
    if (tid < 2) {
        const uint32_t d = tid ? d1 : d0;
        uint32_t lo = d > nb ? d - nb : 0, hi = min(d, na);
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (lt(src[b0 + d - 1 - mid], src[a0 + mid])) hi = mid; else lo = mid + 1;
        }
        split[tid] = lo;
    }
    __syncthreads();
    const uint32_t ia = a0 + split[0], la = split[1] - split[0];
    const uint32_t ib = b0 + (d0 - split[0]), lb = (d1 - d0) - la;
    for (uint32_t i = tid; i < la + lb; i += blockDim.x)
        lds[pidx<SC>(i)] = i < la ? src[ia + i] : src[ib + i - la];
    __syncthreads();
    const uint32_t diag = tid * E;
    const uint32_t tot = la + lb;
    if (diag < tot) {
        const uint32_t x = merge_path<SC>(lds, 0, la, la, lb, diag);
        SC out[E];
        serial_merge<SC, E>(lds, x, la, la + diag - x, tot, tot - 1, out);
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (diag + k < tot) dst[c0 + diag + k] = out[k];
    }
}

// ------------------------------------------------------------------------------ Steps 5-6

// One workgroup per sublist; lane j locates global sample g_j = S[(j+1) m - 1] of the
// sublist's segment: r_ij = #{x : (A_i[x], i*L + x) <= g_j}, a monotone predicate on the
// sorted sublist, found by bisection.  Pads (x >= count) are key-max items.
template <class K, bool V>
__global__ __launch_bounds__(256) void k_rank(const K *keys, const void *sorted_samples,
                                              uint32_t *counts, SegView sv, uint32_t L,
                                              uint32_t s) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    __shared__ uint32_t rk[1025];
    TileLoc loc;
    if (!locate_tile(sv, L, blockIdx.x, loc)) return;
    const uint32_t base = loc.seg_begin + loc.i * L;
    const uint32_t count = min(L, loc.seg_size - loc.i * L);
    const SC *S = (const SC *)sorted_samples + (size_t)loc.tile0 * s;
    const uint32_t p0 = loc.i * L;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        const SC g = S[(size_t)(j + 1) * loc.m - 1];
        uint32_t lo = 0, hi = L;
        while (lo < hi) {
            const uint32_t x = (lo + hi) >> 1;
            const K kx = x < count ? keys[base + x] : KeyMax<K>::v;
            if (!lt(g, R::samp(kx, p0 + x))) lo = x + 1; else hi = x;
        }
        rk[j + 1] = lo;
    }
    if (threadIdx.x == 0) rk[0] = 0;
    __syncthreads();
    uint32_t *row = counts + (size_t)(loc.tile0 + loc.i) * s;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) row[j] = rk[j + 1] - rk[j];
}

// ------------------------------------------------------------------------------ Step 7

// Exclusive scan of v[0, n) in LDS by thread 0 (n <= 1024); returns the total.
__device__ __forceinline__ uint32_t lds_scan_serial(uint32_t *v, uint32_t n) {
    __shared__ uint32_t total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t x = v[j];
            v[j] = run;
            run += x;
        }
        total = run;
    }
    __syncthreads();
    return total;
}

// Writes the bucket table {begin, real size} of one segment and, when asked, the tile map of
// the next level (ceil(size / L_next) per bucket, exclusive prefix, G_next + 1 entries).
// Pads are the largest items, so after Step 8 they fill exactly [seg_size, n') of the
// segment; a bucket's real size is its overlap with [0, seg_size) (several trailing buckets
// may hold pads when the last sublist is mostly padding).
__device__ void emit_buckets(const uint32_t *colsum, const uint32_t *colbase, uint32_t s,
                             uint32_t seg_begin, uint32_t seg_size, uint2 *buckets,
                             uint32_t *tile_off_next, uint32_t L_next, uint32_t *tmp) {
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        const uint32_t b = colbase[j];
        const uint32_t size = b >= seg_size ? 0u : min(colsum[j], seg_size - b);
        buckets[j] = make_uint2(seg_begin + colbase[j], size);
        if (tile_off_next) tmp[j] = (size + L_next - 1) / L_next;
    }
    if (tile_off_next) {
        const uint32_t tot = lds_scan_serial(tmp, s);
        for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) tile_off_next[j] = tmp[j];
        if (threadIdx.x == 0) tile_off_next[s] = tot;
    }
}

// One workgroup per segment (segments with at most a few thousand sublists).
__global__ __launch_bounds__(256) void k_scan_small(const uint32_t *counts, uint32_t *offs,
                                                    SegView sv, uint32_t L, uint32_t s,
                                                    uint2 *buckets, uint32_t *tile_off_next,
                                                    uint32_t L_next) {
    __shared__ uint32_t colsum[1024], colbase[1024], tmp[1024];
    uint32_t tile0, m, seg_begin, seg_size;
    if (!sv.tile_off) {
        tile0 = 0; m = (sv.n_single + L - 1) / L; seg_begin = 0; seg_size = sv.n_single;
    } else {
        tile0 = sv.tile_off[blockIdx.x];
        if (sv.tile_off[blockIdx.x + 1] > sv.max_tiles) return;
        m = sv.tile_off[blockIdx.x + 1] - tile0;
        seg_begin = sv.seg[blockIdx.x].x;
        seg_size = sv.seg[blockIdx.x].y;
    }
    const uint32_t *C = counts + (size_t)tile0 * s;
    uint32_t *O = offs + (size_t)tile0 * s;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t sum = 0;
        for (uint32_t i = 0; i < m; ++i) sum += C[(size_t)i * s + j];
        colsum[j] = sum;
        colbase[j] = sum;
    }
    lds_scan_serial(colbase, s);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t run = seg_begin + colbase[j];
        for (uint32_t i = 0; i < m; ++i) {
            O[(size_t)i * s + j] = run;
            run += C[(size_t)i * s + j];
        }
    }
    emit_buckets(colsum, colbase, s, seg_begin, seg_size, buckets + (size_t)blockIdx.x * s,
                 tile_off_next, L_next, tmp);
}

// Three-kernel form for one large segment [0, n): (a) column sums of each block of RB rows,
// (b) one workgroup scans them per column and across columns, (c) every block writes its
// offsets.
__global__ __launch_bounds__(256) void k_scan_partial(const uint32_t *counts, uint32_t *partial,
                                                      uint32_t m, uint32_t s, uint32_t RB) {
    const uint32_t i0 = blockIdx.x * RB, i1 = min(m, i0 + RB);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t sum = 0;
        for (uint32_t i = i0; i < i1; ++i) sum += counts[(size_t)i * s + j];
        partial[(size_t)blockIdx.x * s + j] = sum;
    }
}

__global__ __launch_bounds__(256) void k_scan_mid(uint32_t *partial, uint32_t nrb, uint32_t s,
                                                  uint32_t n, uint2 *buckets,
                                                  uint32_t *tile_off_next, uint32_t L_next) {
    __shared__ uint32_t colsum[1024], colbase[1024], tmp[1024];
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t run = 0;
        for (uint32_t b = 0; b < nrb; ++b) {
            const uint32_t x = partial[(size_t)b * s + j];
            partial[(size_t)b * s + j] = run;
            run += x;
        }
        colsum[j] = run;
        colbase[j] = run;
    }
    lds_scan_serial(colbase, s);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x)
        for (uint32_t b = 0; b < nrb; ++b) partial[(size_t)b * s + j] += colbase[j];
    emit_buckets(colsum, colbase, s, 0u, n, buckets, tile_off_next, L_next, tmp);
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *counts, const uint32_t *partial,
                                                    uint32_t *offs, uint32_t m, uint32_t s,
                                                    uint32_t RB) {
    const uint32_t i0 = blockIdx.x * RB, i1 = min(m, i0 + RB);
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        uint32_t run = partial[(size_t)blockIdx.x * s + j];
        for (uint32_t i = i0; i < i1; ++i) {
            offs[(size_t)i * s + j] = run;
            run += counts[(size_t)i * s + j];
        }
    }
}

// ------------------------------------------------------------------------------ Step 8

// One workgroup per sorted sublist: item r of piece j (ranks [st_j, st_{j+1})) moves to
// l_ij + r - st_j.  Pads (r >= count) are never written.
template <class K, bool V>
__global__ __launch_bounds__(256) void k_relocate(const K *src, K *dst, const uint32_t *src_vals,
                                                  uint32_t *dst_vals, const uint32_t *counts,
                                                  const uint32_t *offs, SegView sv, uint32_t L,
                                                  uint32_t s) {
    __shared__ uint32_t st[1025], of[1024];
    TileLoc loc;
    if (!locate_tile(sv, L, blockIdx.x, loc)) return;
    const uint32_t base = loc.seg_begin + loc.i * L;
    const uint32_t count = min(L, loc.seg_size - loc.i * L);
    const size_t row = (size_t)(loc.tile0 + loc.i) * s;
    for (uint32_t j = threadIdx.x; j < s; j += blockDim.x) {
        st[j] = counts[row + j];
        of[j] = offs[row + j];
    }
    lds_scan_serial(st, s);
    for (uint32_t r = threadIdx.x; r < count; r += blockDim.x) {
        uint32_t lo = 0, hi = s - 1;  // largest j with st[j] <= r
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (st[mid] <= r) lo = mid; else hi = mid - 1;
        }
        const uint32_t d = of[lo] + (r - st[lo]);
        if (d >= sv.n_total) continue;  // defensive: offsets always lie inside the array
        dst[d] = src[base + r];
        if (V) dst_vals[d] = src_vals[base + r];
    }
}

// ------------------------------------------------------------------------------ misc

__global__ void k_init(uint32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = 0;
}

// ------------------------------------------------------------------------------ host driver

#define DS_CHECK_LAUNCH()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return DSORT_E_HIP; \
    } while (0)

// Launch with optional timing events around it.
#define DS_LAUNCH(NAME, KERNEL, GRID, BLOCK, ...)                                   \
    do {                                                                            \
        void *ev1_ = nullptr;                                                       \
        if (tm && stage_begin(*tm, NAME, st, &ev1_) != DSORT_OK) return DSORT_E_HIP; \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, st, __VA_ARGS__);                \
        if (hipGetLastError() != hipSuccess) return DSORT_E_HIP;                    \
        if (ev1_ && hipEventRecord((hipEvent_t)ev1_, st) != hipSuccess) return DSORT_E_HIP; \
    } while (0)

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

template <class K, bool V, bool F32> struct Pipeline {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    static constexpr int TE = (sizeof(typename R::T) >= 16) ? 8 : 16;  // Step 2 items/thread
    static constexpr int TCAP = TE * 1024;                            // largest L
    static constexpr int FE = (!V && sizeof(K) == 4) ? 32 : TE;       // Step 9 items/thread
    static constexpr int FCAP = FE * 1024;                            // bucket capacity
    static constexpr int SE = sizeof(SC) >= 16 ? 8 : 16;
    static constexpr int SCAP = SE * 1024;

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
            DS_LAUNCH(name_merge, (k_merge_round<SC, SE, SCAP>), dim3(chunks), dim3(SCAP / SE),
                      (const SC *)x, y, total, run);
            SC *t = x;
            x = y;
            y = t;
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
        uint2 *buckets1 = (uint2 *)(ws + g.o_buckets1);
        uint32_t *tileoff2 = g.levels == 2 ? (uint32_t *)(ws + g.o_tileoff2) : nullptr;
        const SegView sv1{nullptr, nullptr, 1, n, n, g.m1};

        // Steps 1-3
        {
            TileArgs a{keys, keys, d_vals, d_vals, sv1, g.L1, g.s1, samp, status};
            DS_LAUNCH("s123_local_sort", (k_tile<K, V, TE, TCAP, MODE_SAMPLE, F32, false>),
                      dim3(g.m1), dim3(g.L1 / TE), a);
        }
        // Step 4
        int rc = sort_samples(samp, sorted, tmp, sv1, g.L1, g.s1, 1, g.m1 * g.s1, status, st,
                              g.samp_global, g.samp_rounds, tm, "s4_sample_sort",
                              "s4_sample_merge");
        if (rc) return rc;
        // Steps 5-6
        DS_LAUNCH("s56_rank", (k_rank<K, V>), dim3(g.m1), dim3(256), (const K *)keys,
                  (const void *)sorted, counts, sv1, g.L1, g.s1);
        // Step 7
        if (!g.scan_large) {
            DS_LAUNCH("s7_scan", k_scan_small, dim3(1), dim3(256), (const uint32_t *)counts,
                      offs, sv1, g.L1, g.s1, buckets1, tileoff2, g.L2);
        } else {
            uint32_t *partial = (uint32_t *)(ws + g.o_partial);
            DS_LAUNCH("s7_scan_colsum", k_scan_partial, dim3(g.scan_nrb), dim3(256),
                      (const uint32_t *)counts, partial, g.m1, g.s1, g.scan_rb);
            DS_LAUNCH("s7_scan_mid", k_scan_mid, dim3(1), dim3(256), partial, g.scan_nrb, g.s1,
                      n, buckets1, tileoff2, g.L2);
            DS_LAUNCH("s7_scan_update", k_scan_apply, dim3(g.scan_nrb), dim3(256),
                      (const uint32_t *)counts, (const uint32_t *)partial, offs, g.m1, g.s1,
                      g.scan_rb);
        }
        // Step 8
        DS_LAUNCH("s8_relocate", (k_relocate<K, V>), dim3(g.m1), dim3(256), (const K *)keys,
                  wkeys, (const uint32_t *)d_vals, wvals, (const uint32_t *)counts,
                  (const uint32_t *)offs, sv1, g.L1, g.s1);

        if (g.levels == 1) {
            // Step 9: every bucket in one workgroup, from the relocated copy back into keys.
            TileArgs a{wkeys, keys, wvals, d_vals, SegView{buckets1, nullptr, g.s1, 0, n, 0}, 0,
                       0, nullptr, status};
            DS_LAUNCH("s9_bucket_sort", (k_tile<K, V, FE, FCAP, MODE_FINAL, false, F32>),
                      dim3(g.s1), dim3(FCAP / FE), a);
            return DSORT_OK;
        }

        // Step 9 as a second level: Algorithm 1 on every bucket of level 1.
        const SegView sv2{buckets1, tileoff2, g.s1, 0, n, g.tiles2max};
        SC *samp2 = (SC *)(ws + g.o_samp2);
        SC *sorted2 = (SC *)(ws + g.o_samp2_sorted);
        uint32_t *counts2 = (uint32_t *)(ws + g.o_counts2);
        uint32_t *offs2 = (uint32_t *)(ws + g.o_offs2);
        uint2 *finals = (uint2 *)(ws + g.o_final);
        {
            TileArgs a{wkeys, wkeys, wvals, wvals, sv2, g.L2, g.s2, samp2, status};
            DS_LAUNCH("l2_s123_local_sort", (k_tile<K, V, TE, TCAP, MODE_SAMPLE, false, false>),
                      dim3(g.tiles2max), dim3(g.L2 / TE), a);
        }
        rc = sort_samples(samp2, sorted2, nullptr, sv2, g.L2, g.s2, g.s1, 0, status, st, false, 0,
                          tm, "l2_s4_sample_sort", "l2_s4_sample_merge");
        if (rc) return rc;
        DS_LAUNCH("l2_s56_rank", (k_rank<K, V>), dim3(g.tiles2max), dim3(256), (const K *)wkeys,
                  (const void *)sorted2, counts2, sv2, g.L2, g.s2);
        DS_LAUNCH("l2_s7_scan", k_scan_small, dim3(g.s1), dim3(256), (const uint32_t *)counts2,
                  offs2, sv2, g.L2, g.s2, finals, (uint32_t *)nullptr, 0u);
        DS_LAUNCH("l2_s8_relocate", (k_relocate<K, V>), dim3(g.tiles2max), dim3(256),
                  (const K *)wkeys, keys, (const uint32_t *)wvals, d_vals,
                  (const uint32_t *)counts2, (const uint32_t *)offs2, sv2, g.L2, g.s2);
        {
            TileArgs a{keys, keys, d_vals, d_vals, SegView{finals, nullptr, g.final_buckets, 0, n, 0},
                       0, 0, nullptr, status};
            DS_LAUNCH("s9_bucket_sort", (k_tile<K, V, FE, FCAP, MODE_FINAL, false, F32>),
                      dim3(g.final_buckets), dim3(FCAP / FE), a);
        }
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

int run_pipeline(const Geom &g, void *d_keys, uint32_t *d_vals, void *d_ws, void *stream,
                 Timing *tm) {
    hipStream_t st = (hipStream_t)stream;
    if (g.levels < 0) return DSORT_OK;
    if (g.n > 0xFFFFFFFFull) return DSORT_E_INVALID;
    if (tm && !tm->enabled) tm = nullptr;
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

}  // namespace dsort
