// The kernels of Algorithm 1's steps (gfx950): Steps 1-3 and the one-tile sort (k_tile),
// Step 4 (k_sort_samples, k_merge_round), Steps 5-6 (k_rank), Step 7 (the scans), Steps
// 8-9 fused (k_gather_bsort), and the set-up, relocation and copy kernels.  Included once,
// by kernels.hip.
#pragma once

#include "sort_primitives.h"

namespace dsort {
namespace {

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
    void *rank_idx;        // MODE_SAMPLE, optional: L/16 keys per tile, the key at rank 16q+15
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
        // eight rows of the wave's share per pass: their loads are in flight together.  The
        // lane's piece end and source offset stay in registers until it enters the next piece.
        uint32_t pend = tb[p + 1], soff = sb[p];
        for (uint32_t row = xs; row < xe; row += 8 * wl) {
            uint32_t si[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t xu = row + wl * u + lane;
                if (xu < xe) {
                    while (xu >= pend) {
                        ++p;
                        pend = tb[p + 1];
                        soff = sb[p];
                    }
                    si[u] = soff + xu;
                }
            }
            store.template run<8>(row + lane, wl, xe, si);
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
// Keys-only 32-bit tiles of 1024 threads ask for eight waves per SIMD (at most 64 VGPRs), which
// two resident workgroups per CU need.
template <class K, bool V, int E, int CAP>
constexpr int tile_waves_per_eu() { return !V && sizeof(K) == 4 && CAP / E == 1024 ? 8 : 1; }

// 128-bit loads and stores of a tile's keys (four 32-bit or two 64-bit keys per access): for
// whole tiles (count = P = E * blockDim, E a multiple of the keys per access) whose keys start
// on a 16-byte boundary.  The keys of one access never straddle an LDS pad.
template <class K> struct Vec16 {
    static constexpr int n = 16 / (int)sizeof(K);
    static __device__ __forceinline__ void unpack(const uint4 &v, K (&k)[16 / sizeof(K)]) {
        if constexpr (sizeof(K) == 4) {
            k[0] = v.x; k[1] = v.y; k[2] = v.z; k[3] = v.w;
        } else {
            k[0] = ((uint64_t)v.y << 32) | v.x;
            k[1] = ((uint64_t)v.w << 32) | v.z;
        }
    }
    static __device__ __forceinline__ uint4 pack(const K (&k)[16 / sizeof(K)]) {
        if constexpr (sizeof(K) == 4) {
            return make_uint4(k[0], k[1], k[2], k[3]);
        } else {
            return make_uint4((uint32_t)k[0], (uint32_t)(k[0] >> 32), (uint32_t)k[1],
                              (uint32_t)(k[1] >> 32));
        }
    }
};
template <class K, int E>
__device__ __forceinline__ bool tile_vec4(const K *p, uint32_t count, uint32_t P) {
    return E % Vec16<K>::n == 0 && count == P && P == E * blockDim.x && ((uintptr_t)p & 15) == 0;
}

template <class K, bool V, int E, int CAP, int MODE, bool XIN, bool XOUT, bool GIN = false>
__global__ __launch_bounds__(CAP / E, (tile_waves_per_eu<K, V, E, CAP>())) void k_tile(TileArgs a) {
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
    } else if (tile_vec4<K, E>(src + begin, count, P)) {
        // whole tile, 16-byte aligned: 128-bit loads, consecutive lanes on consecutive 16-byte
        // words, all of a thread's loads in flight together
        constexpr int NV = Vec16<K>::n;
        uint4 v[E / NV];
        const uint4 *s4 = (const uint4 *)(src + begin);
#pragma unroll
        for (int q = 0; q < E / NV; ++q) v[q] = s4[tid + q * bd];
#pragma unroll
        for (int q = 0; q < E / NV; ++q) {
            const uint32_t i = NV * (tid + q * bd);
            T *d = lds + pidx<T>(i);
            K w[NV];
            Vec16<K>::unpack(v[q], w);
#pragma unroll
            for (int r = 0; r < NV; ++r)
                d[r] = R::make(XIN ? (K)f32_in((uint32_t)w[r]) : w[r], i + r);
        }
    } else {
        // P <= E * blockDim.x: every thread's E loads are issued before any is waited for
        K v[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * bd;
            v[q] = i < count ? src[begin + i] : KeyMax<K>::v;
        }
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * bd;
            if (i < P) {
                K k = v[q];
                if (XIN) k = (K)f32_in((uint32_t)k);
                lds[pidx<T>(i)] = i < count ? R::make(k, i) : R::pad(i);
            }
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
    if (tile_vec4<K, E>(dst + begin, count, P)) {
        constexpr int NV = Vec16<K>::n;
        uint4 *d4 = (uint4 *)(dst + begin);
#pragma unroll 2
        for (int q = 0; q < E / NV; ++q) {
            const uint32_t i = NV * (tid + q * bd);
            const T *l = lds + pidx<T>(i);
            K w[NV];
#pragma unroll
            for (int r = 0; r < NV; ++r) {
                const K k = R::key(l[r]);
                w[r] = XOUT ? (K)f32_out((uint32_t)k) : k;
            }
            d4[tid + q * bd] = Vec16<K>::pack(w);
        }
    } else {
#pragma unroll 2
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * bd;
            if (i < count) {
                K k = R::key(lds[pidx<T>(i)]);
                if (XOUT) k = (K)f32_out((uint32_t)k);
                dst[begin + i] = k;
            }
        }
    }
    if (MODE == MODE_SAMPLE && a.rank_idx) {
        // the rank index of Steps 5-6: every 16th key of the sorted sublist (pads: key-max)
        K *ix = (K *)a.rank_idx + (size_t)(loc.tile0 + loc.i) * (a.L / 16);
        for (uint32_t q = tid; q < a.L / 16; q += bd) ix[q] = R::key(lds[pidx<T>(16 * q + 15)]);
    }
    if constexpr (V) {
        __syncthreads();
        if (GIN)
            tile_gather(a.pdst + loc.piece0, a.psrc + loc.piece0, loc.seg_begin, loc.i * a.L,
                        count, p_first, p_last, tb, sb,
                        GatherVals<T>{a.src_vals, lds, a.sv.n_total});
        else
        {
            uint32_t vv[E];
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const uint32_t i = tid + q * bd;
                vv[q] = i < count ? a.src_vals[begin + i] : 0u;
            }
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const uint32_t i = tid + q * bd;
                if (i < count) put_val<T>(lds, i, vv[q]);
            }
        }
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
    {  // P <= E * blockDim.x: all of a thread's loads in flight together
        SC v[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * blockDim.x;
            v[q] = i < count ? src[begin + i] : MaxOf<SC>::get();
        }
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const uint32_t i = tid + q * blockDim.x;
            if (i < P) lds[pidx<SC>(i)] = v[q];
        }
    }
    __syncthreads();
    // Each sublist's s samples are already in order (they come from its sorted items), and
    // every range starts on a row (a segment's) or at a multiple of CAP (fixed chunks), so the
    // sort starts from the aligned runs of the largest power of two r dividing s: no row
    // boundary falls inside one.  Sample composites are in position order.
    const uint32_t r = s & (0u - s);
    block_sort<SC, E, true>(lds, P, r > (uint32_t)E ? r : (uint32_t)E);
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
// together (chunks shared by neighbouring samples come from cache); chunks of at most 16
// items take four samples per wave load, one per 16-lane group.  Chunks of 128 to 1024 items
// read a rank index instead when the tile sort wrote one (rank_blocks); other large chunks are
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

// The chunk counts for chunks of at most 16 items: each 16-lane group of a wave takes its own
// global sample, so one load instruction covers four samples' chunks (kRankBatch loads in
// flight per lane: 4 kRankBatch samples per wave and batch).
template <class K, bool V>
__device__ __forceinline__ void rank_chunks16(const K *keys, const typename Tr<K, V>::SC *S,
                                              uint32_t m, const uint32_t *chunk, uint32_t *rk,
                                              uint32_t s, uint32_t w, uint32_t base,
                                              uint32_t count, uint32_t p0) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    const uint32_t lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = lane >> 4, y = lane & 15;
    constexpr uint32_t kB = 4 * kRankBatch;  // samples per wave and batch
    for (uint32_t j0 = wv * kB; j0 < s; j0 += nwv * kB) {
        K v[kRankBatch];
        uint32_t cc[kRankBatch];
        SC gg[kRankBatch];
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t j = j0 + 4 * u + g;  // this lane group's sample
            cc[u] = j < s ? chunk[j] : s;
            gg[u] = cc[u] < s ? S[(size_t)(j + 1) * m - 1] : SC{};
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t x = cc[u] * w + y;
            v[u] = (cc[u] < s && y < w && x < count) ? keys[base + x] : KeyMax<K>::v;
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t c = cc[u];
            const bool in = c < s && y < w && !lt(gg[u], R::samp(v[u], p0 + c * w + y));
            const uint64_t bits = __ballot(in) >> (16 * g);
            const uint32_t le = (uint32_t)__popcll(bits & 0xFFFFull);
            if (c < s && y == 0) rk[j0 + 4 * u + g + 1] = c * w + le;
        }
    }
}

// The same counts through the rank index (every 16th key of each sorted sublist, at rank
// 16q + 15): per global sample, one lane per index entry of its chunk counts the entries <= g_j
// (each is the largest item of its block of 16, so that many whole blocks precede the rank),
// then 16 lanes count inside the one block that holds the rank.  About 16 + w/4 bytes per
// (sublist, splitter) pair are read instead of 4w (32-bit keys).  w = 16 nb, nb <= 64 (chunks
// of at most 16 blocks take rank_blocks16).
template <class K, bool V>
__device__ __forceinline__ void rank_blocks(const K *keys, const K *ix,
                                            const typename Tr<K, V>::SC *S, uint32_t m,
                                            const uint32_t *chunk, uint32_t *rk, uint32_t s,
                                            uint32_t w, uint32_t base, uint32_t count,
                                            uint32_t p0) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    const uint32_t lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nb = w / 16;
    for (uint32_t j0 = wv * kRankBatch; j0 < s; j0 += nwv * kRankBatch) {
        K v[kRankBatch];
        uint32_t cc[kRankBatch];
        SC gg[kRankBatch];
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            cc[u] = j0 + u < s ? __builtin_amdgcn_readfirstlane(chunk[j0 + u]) : s;
            gg[u] = cc[u] < s ? S[(size_t)(j0 + u + 1) * m - 1] : SC{};
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u)
            v[u] = (cc[u] < s && lane < nb) ? ix[cc[u] * nb + lane] : KeyMax<K>::v;
        uint32_t bb[kRankBatch];  // blocks wholly <= g_j (wave-uniform)
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const bool in = lane < nb && !lt(gg[u], R::samp(v[u], p0 + cc[u] * w + 16 * lane + 15));
            bb[u] = (uint32_t)__popcll(__ballot(in));
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t x = cc[u] * w + 16 * bb[u] + lane;
            v[u] = (cc[u] < s && lane < 16 && x < count) ? keys[base + x] : KeyMax<K>::v;
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t c = cc[u];
            if (c >= s) continue;
            const uint32_t x0 = c * w + 16 * bb[u];
            const bool in = lane < 16 && !lt(gg[u], R::samp(v[u], p0 + x0 + lane));
            const uint32_t le = (uint32_t)__popcll(__ballot(in));
            if (lane == 0) rk[j0 + u + 1] = x0 + le;
        }
    }
}

// rank_blocks for chunks of 4 to 16 index entries (64 <= w <= 256): each 16-lane group of a
// wave takes its own global sample, so one load instruction serves four samples in both phases
// (at 2^28 u32: level-1 ranks, 64-item chunks, 0.29 -> 0.16 ms; level-2 ranks, 128-item
// chunks, 0.18 -> 0.11 ms).
template <class K, bool V>
__device__ __forceinline__ void rank_blocks16(const K *keys, const K *ix,
                                              const typename Tr<K, V>::SC *S, uint32_t m,
                                              const uint32_t *chunk, uint32_t *rk, uint32_t s,
                                              uint32_t w, uint32_t base, uint32_t count,
                                              uint32_t p0) {
    using R = Tr<K, V>;
    using SC = typename R::SC;
    const uint32_t lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = lane >> 4, y = lane & 15;
    const uint32_t nb = w / 16;
    constexpr uint32_t kB = 4 * kRankBatch;  // samples per wave and batch
    for (uint32_t j0 = wv * kB; j0 < s; j0 += nwv * kB) {
        K v[kRankBatch];
        uint32_t cc[kRankBatch], bb[kRankBatch];
        SC gg[kRankBatch];
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t j = j0 + 4 * u + g;  // this lane group's sample
            cc[u] = j < s ? chunk[j] : s;
            gg[u] = cc[u] < s ? S[(size_t)(j + 1) * m - 1] : SC{};
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u)
            v[u] = (cc[u] < s && y < nb) ? ix[cc[u] * nb + y] : KeyMax<K>::v;
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const bool in = cc[u] < s && y < nb &&
                            !lt(gg[u], R::samp(v[u], p0 + cc[u] * w + 16 * y + 15));
            bb[u] = (uint32_t)__popcll((__ballot(in) >> (16 * g)) & 0xFFFFull);
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t x = cc[u] * w + 16 * bb[u] + y;
            v[u] = (cc[u] < s && x < count) ? keys[base + x] : KeyMax<K>::v;
        }
#pragma unroll
        for (uint32_t u = 0; u < kRankBatch; ++u) {
            const uint32_t c = cc[u], x0 = c * w + 16 * bb[u];
            const bool in = c < s && !lt(gg[u], R::samp(v[u], p0 + x0 + y));
            const uint32_t le = (uint32_t)__popcll((__ballot(in) >> (16 * g)) & 0xFFFFull);
            if (c < s && y == 0) rk[j0 + 4 * u + g + 1] = x0 + le;
        }
    }
}

template <class K, bool V>
__global__ __launch_bounds__(256) void k_rank(const K *keys, const void *sorted_samples,
                                              const void *tile_samples, uint32_t *counts,
                                              SegView sv, uint32_t L, uint32_t s,
                                              uint32_t random, const K *rank_idx) {
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
    if (rank_idx && w % 16 == 0 && w >= 64 && w <= 256) {
        rank_blocks16<K, V>(keys, rank_idx + (size_t)(loc.tile0 + loc.i) * (L / 16), S, loc.m,
                            chunk, rk, s, w, base, count, p0);
    } else if (rank_idx && w % 16 == 0 && w > 256 && w <= 1024) {
        rank_blocks<K, V>(keys, rank_idx + (size_t)(loc.tile0 + loc.i) * (L / 16), S, loc.m,
                          chunk, rk, s, w, base, count, p0);
    } else if (w <= 16) {
        rank_chunks16<K, V>(keys, S, loc.m, chunk, rk, s, w, base, count, p0);
    } else if (w <= 64) {
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
    // s <= blockDim: ng groups of s threads; the threads past the last whole group only join
    // the barriers
    const uint32_t ng = blockDim.x / s;
    const uint32_t grp = threadIdx.x / s, j = threadIdx.x % s;
    const bool live = grp < ng;
    const uint32_t per = (nrb + ng - 1) / ng;
    const uint32_t b0 = live ? min(nrb, grp * per) : nrb, b1 = live ? min(nrb, b0 + per) : nrb;
    uint32_t own = 0;
#pragma unroll 8
    for (uint32_t b = b0; b < b1; ++b) own += partial[(size_t)b * s + j];
    if (live) tmp[grp * s + j] = own;
    __syncthreads();
    uint32_t run = 0;
    for (uint32_t q = 0; live && q < grp; ++q) run += tmp[q * s + j];
    if (live && grp == ng - 1) {
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
            // the lane's piece end and source offset (mod 2^32) stay in registers until it
            // enters the next piece
            uint32_t pend = bnd[p + 1], soff = ps[p] - bnd[p];
            for (uint32_t row = x_begin; row < x_end; row += 4 * 64) {
                K v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t xu = row + 64 * u + lane;
                    if (xu < total) {
                        while (xu >= pend) {
                            ++p;
                            pend = bnd[p + 1];
                            soff = ps[p] - bnd[p];
                        }
                        v[u] = src[soff + xu];
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
            // values by the keys' gather pattern: each wave streams its share of the bucket,
            // every lane following the piece its item is in (whole waves busy even where the
            // pieces are shorter than a wave)
            const uint32_t span = ((total + nw - 1) / nw + 63) & ~63u;
            const uint32_t x_begin = w * span, x_end = min(total, x_begin + span);
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
                uint32_t pend = bnd[p + 1], soff = ps[p] - bnd[p];
                for (uint32_t row = x_begin; row < x_end; row += 4 * 64) {
                    uint32_t vv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t xu = row + 64 * u + lane;
                        if (xu < x_end) {
                            while (xu >= pend) {
                                ++p;
                                pend = bnd[p + 1];
                                soff = ps[p] - bnd[p];
                            }
                            vv[u] = a.src_vals[soff + xu];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const uint32_t xu = row + 64 * u + lane;
                        if (xu < x_end) put_val<T>(lds, xu, vv[u]);
                    }
                }
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

}  // namespace
}  // namespace dsort
