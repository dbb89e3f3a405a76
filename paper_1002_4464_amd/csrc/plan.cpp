// Host side of the C ABI: argument checking, the choice of (L, s) per level, and the
// workspace map.  No HIP runtime call happens here, so all of it runs without a GPU.
//
// Sizes follow Section 4 of the paper: m = ceil(n/L) sublists of L items, s samples per
// sublist, and after Step 8 buckets B_j with m <= |B_j| <= 2n'/s - m (n' = mL, the padded
// size), which is the exact form of the paper's "at most 2n/s" bound under the total order
// (key, sublist, rank).  Every bucket that Step 9 hands to one workgroup must therefore obey
// 2n'/s - m <= capacity, which fixes the smallest admissible s.  When that s would make the
// sample set too large (more than 1/32 of the data), Step 9 instead runs Algorithm 1 again on
// each bucket (a second level), whose buckets then fit one workgroup.
#include <algorithm>
#include <new>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dsort_internal.h"

namespace dsort {

namespace {

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Largest bucket Step 8 can produce with m sublists of L items and s samples per sublist.
uint64_t bucket_bound(uint64_t m, uint64_t L, uint64_t s) { return 2 * m * L / s - m; }

constexpr uint32_t kScanRowBlock = 32;
constexpr uint64_t kMaxSamples = 1024;  // per-sublist tables live in LDS
constexpr uint64_t kMaxPieces = 256;    // pieces per bucket the fused Steps 8-9 accept
constexpr uint64_t kNumClasses = 8;     // size classes of the fused Steps 8-9

// A level's sublist length: a power of two, or a multiple of 64 items per thread (the tile
// kernel then runs whole waves); its sample count divides it (Step 3's chunks of L/s items).
bool level_L_ok(const Caps &c, uint64_t L) {
    return L >= c.tile_e && L <= c.tile_max && (is_pow2(L) || L % (64 * (uint64_t)c.tile_e) == 0);
}
bool level_s_ok(uint64_t s, uint64_t L) { return s && s <= L && s <= kMaxSamples && L % s == 0; }

// Chunks of L/s items that the rank index serves: whole blocks of 16, at least 4 and at most
// 64 of them (one lane per index entry; up to 16 entries, four samples share a wave load).
// Smaller chunks are read whole.
bool rank_index_ok(uint64_t L, uint64_t s) {
    const uint64_t w = L / s;
    return w % 16 == 0 && w >= 64 && w <= 1024;
}

}  // namespace

Caps caps_for(int key_type, bool values) {
    Caps c{};
    if (key_type == DSORT_U64) {
        c.key_bytes = 8;
        c.samp_bytes = 16;
        c.samp_cap = 8192;
        c.samp_e = 8;
        if (values) {
            c.tile_max = 8192; c.tile_e = 8;
            c.final_cap = 8192; c.final_e = 8;
        } else {
            c.tile_max = 16384; c.tile_e = 16;
            c.final_cap = 16384; c.final_e = 16;
        }
    } else {
        c.key_bytes = 4;
        c.samp_bytes = 8;
        c.samp_cap = 16384;
        c.samp_e = 16;
        if (values) {
            c.tile_max = 16384; c.tile_e = 16;
            c.final_cap = 16384; c.final_e = 16;
        } else {
            c.tile_max = 16384; c.tile_e = 16;
            c.final_cap = 32768; c.final_e = 32;
        }
    }
    return c;
}

int make_geom(int key_type, bool values, uint64_t n, const dsort_tuning_t &tu, Geom &g) {
    g = Geom{};
    g.key_type = key_type;
    g.values = values;
    g.n = n;
    g.caps = caps_for(key_type, values);
    const Caps &c = g.caps;
    g.o_status = 0;
    size_t off = 256;
    if (n <= 1) {
        g.levels = -1;
        g.total = off;
        return DSORT_OK;
    }
    const bool tuned = tu.sublist_len || tu.samples || tu.sublist_len2 || tu.samples2 || tu.levels;
    if (tu.levels > 2 || tu.sampling > 1) return DSORT_E_UNSUPPORTED;
    if (!tuned && n <= c.final_cap) {
        g.levels = 0;
        g.total = off;
        return DSORT_OK;
    }

    const uint64_t L1 = tu.sublist_len ? tu.sublist_len : c.tile_max;
    if (!level_L_ok(c, L1)) return DSORT_E_UNSUPPORTED;
    if (tu.samples && !level_s_ok(tu.samples, L1)) return DSORT_E_UNSUPPORTED;
    const uint64_t m1 = ceil_div(n, L1);
    if (m1 * L1 > kMaxItems + L1) return DSORT_E_UNSUPPORTED;

    // --- one level: the smallest s whose bucket bound fits one workgroup.
    uint64_t s1 = 0;
    bool one = false;
    if (tu.levels == 1 && m1 > kMaxPieces) return DSORT_E_UNSUPPORTED;
    if (tu.levels != 2 && m1 <= kMaxPieces) {
        if (tu.samples) {
            s1 = tu.samples;
            one = bucket_bound(m1, L1, s1) <= c.final_cap;
            if (!one && tu.levels == 1) return DSORT_E_UNSUPPORTED;
        } else {
            uint64_t smax = tu.levels == 1 ? L1 : L1 / 32;
            if (smax > kMaxSamples) smax = kMaxSamples;
            for (uint64_t s = 1; s <= smax; s <<= 1)
                if (bucket_bound(m1, L1, s) <= c.final_cap) { s1 = s; one = true; break; }
            if (!one && tu.levels == 1) return DSORT_E_UNSUPPORTED;
        }
    }

    uint64_t L2 = 0, s2 = 0, m2max = 0;
    if (!one) {
        // --- two levels: the smallest s1 for which every bucket can be sorted by one more
        // level whose samples fit one workgroup (Step 4 of the second level stays local).
        L2 = tu.sublist_len2 ? tu.sublist_len2 : c.tile_max;
        if (!level_L_ok(c, L2)) return DSORT_E_UNSUPPORTED;
        if (tu.samples2 && !level_s_ok(tu.samples2, L2)) return DSORT_E_UNSUPPORTED;
        // Untuned choices prefer (measured at 2^25 to 2^28, 32-bit keys with and without values:
        // up to 5 % faster than the smallest feasible s1 and s2) s1 >= n / 2^19, capped at 256
        // (about 32 level-2 sublists per level-1 bucket; more samples, e.g. s1 = 512 at 2^28,
        // cost more in Steps 4-7 than they save), and s2 >= n / (4096 s1), capped at 128 (final
        // buckets of about 4K items, eight merge passes), as long as the level-2 samples still
        // fit one workgroup.  Where no s1 allows that, the smallest feasible s1 and s2.  Under
        // each of the two rules s1 and s2 only grow with n (the workspace walk of dsort_plan
        // relies on that; the rule is part of its piece key).
        const uint64_t hi = tu.samples ? tu.samples : (L1 / 8 < kMaxSamples ? L1 / 8 : kMaxSamples);
        const uint64_t t_lo = tu.samples2 ? tu.samples2 : 1;
        const uint64_t t_hi = tu.samples2 ? tu.samples2 : (L2 < kMaxSamples ? L2 : kMaxSamples);
        auto search = [&](bool pref) {
            uint64_t p1 = 2;
            while (pref && p1 < 256 && p1 < (n >> 19)) p1 <<= 1;
            for (uint64_t s = tu.samples ? tu.samples : p1; s <= hi; s <<= 1) {
                const uint64_t mm = ceil_div(bucket_bound(m1, L1, s), L2);
                if (mm > kMaxPieces) continue;
                uint64_t t = t_lo;  // smallest s2 whose buckets fit one workgroup
                while (t <= t_hi && mm * (2 * L2 / t - 1) > c.final_cap) t <<= 1;
                if (t > t_hi) continue;
                if (pref && !tu.samples2)
                    while (t < 128 && t < t_hi && t * s * 4096 < n) t <<= 1;
                if (mm * t > c.samp_cap) continue;
                s1 = s; s2 = t; m2max = mm;
                return true;
            }
            return false;
        };
        const bool found = search(true) || (g.plan_rule = 1, search(false));
        if (!found) return DSORT_E_UNSUPPORTED;
    }

    g.L1 = (uint32_t)L1;
    g.s1 = (uint32_t)s1;
    g.m1 = (uint32_t)m1;
    g.beta1 = (uint32_t)bucket_bound(m1, L1, s1);
    const uint64_t sm = m1 * s1;
    g.samp_global = sm > c.samp_cap;
    if (g.samp_global) {
        uint32_t r = 0;
        for (uint64_t run = c.samp_cap; run < sm; run <<= 1) ++r;
        g.samp_rounds = r;
    }
    g.scan_large = true;
    g.scan_rb = kScanRowBlock;
    g.scan_nrb = (uint32_t)ceil_div(m1, kScanRowBlock);

    if (one) {
        g.levels = 1;
        g.final_buckets = (uint32_t)s1;
    } else {
        g.levels = 2;
        g.L2 = (uint32_t)L2;
        g.s2 = (uint32_t)s2;
        g.m2max = (uint32_t)m2max;
        g.tiles2max = (uint32_t)(ceil_div(n, L2) + s1);
        g.final_buckets = (uint32_t)(s1 * s2);
    }
    if (tu.sampling == 1) {
        // Randomized samples bound no bucket.  The normal path takes a level-1 bucket of up to
        // one workgroup (one level), or of as many level-2 sublists as the level-2 sample sort
        // and bucket capacity allow with this s2 (two levels; the level-2 grid, ceil(n/L2) + s1
        // tiles, covers any split of n into s1 buckets).
        g.random = true;
        g.seed = tu.seed;
        if (one) {
            g.bucket_limit = c.final_cap;
        } else {
            uint64_t mm = 0;
            while (mm < kMaxPieces && (mm + 1) * s2 <= c.samp_cap &&
                   bucket_bound(mm + 1, L2, s2) <= c.final_cap)
                ++mm;
            g.bucket_limit = (uint32_t)std::min<uint64_t>(mm * L2, 0xFFFFFFFFull);
        }
    }

    // --- workspace map
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    g.o_wkeys = take(n * c.key_bytes);
    if (values) g.o_wvals = take(n * 4);
    g.o_samp = take(sm * c.samp_bytes);
    g.o_samp_sorted = take(sm * c.samp_bytes);
    if (g.samp_global) g.o_samp_tmp = take(sm * c.samp_bytes);
    g.o_counts = take(sm * 4);
    g.o_offs = take(sm * 4);
    g.o_pdst = take(sm * 4);
    g.o_psrc = take(sm * 4);
    g.o_partial = take((size_t)g.scan_nrb * s1 * 4);
    g.o_buckets1 = take(s1 * 16);
    if (g.levels == 2) {
        g.o_tileoff2 = take((s1 + 1) * 4);
        const size_t sm2 = (size_t)g.tiles2max * s2;
        g.o_samp2 = take(sm2 * c.samp_bytes);
        g.o_samp2_sorted = take(sm2 * c.samp_bytes);
        g.o_counts2 = take(sm2 * 4);
        g.o_offs2 = take(sm2 * 4);
        g.o_pdst2 = take(sm2 * 4);
        g.o_psrc2 = take(sm2 * 4);
        g.o_final = take((size_t)g.final_buckets * 16);
    } else {
        g.o_final = g.o_buckets1;
    }
    g.o_lists = take((size_t)kNumClasses * g.final_buckets * 4);
    if (g.random) g.o_ovf = take(s1 * 4);
    // Steps 5-6 read a chunk's index entries, then one block of 16 items, when the chunks are
    // whole blocks of at least two (chunk-end samples; the randomized ranks bisect instead)
    if (!g.random && rank_index_ok(L1, s1)) g.o_idx1 = take(m1 * (L1 / 16) * c.key_bytes);
    if (g.levels == 2 && rank_index_ok(L2, s2))
        g.o_idx2 = take((size_t)g.tiles2max * (L2 / 16) * c.key_bytes);
    g.total = off;
    return DSORT_OK;
}

// Segmented sorts (one level per long segment).  A segment of z > small_cap items has
// m = ceil(z/L) sublists; its s must keep every bucket within one workgroup
// (m (2L/s - 1) <= final_cap, the bound of Section 4) and its m*s samples within the
// one-workgroup sample sort (<= samp_cap).
uint64_t seg_samples(const Caps &c, uint64_t m, uint64_t L) {
    if (m == 0 || m > kMaxPieces) return 0;
    for (uint64_t s = 1; s <= L && s <= kMaxSamples; s <<= 1)
        if (bucket_bound(m, L, s) <= c.final_cap) return m * s <= c.samp_cap ? s : 0;
    return 0;
}

static bool seg_L_ok(const Caps &c, uint64_t L) {
    return is_pow2(L) && L <= c.tile_max && L >= 64 * (uint64_t)c.tile_e;
}

int seg_candidate_L(const Caps &c, uint32_t *out) {
    int k = 0;
    for (uint64_t L = c.tile_max; k < 4 && seg_L_ok(c, L); L >>= 1) out[k++] = (uint32_t)L;
    return k;
}

uint64_t seg_limit(int key_type, bool values) {
    const Caps c = caps_for(key_type, values);
    uint64_t m = 1;
    while (m < kMaxPieces && seg_samples(c, m + 1, c.tile_max)) ++m;
    const uint64_t lim = seg_samples(c, m, c.tile_max) ? m * c.tile_max : 0;
    return lim > c.final_cap ? lim : c.final_cap;
}

static uint64_t clamp_max_seg(uint64_t n, uint64_t max_seg, uint64_t lim) {
    if (max_seg == 0) max_seg = n < lim ? n : lim;
    return max_seg > n ? n : max_seg;
}

SegTuning seg_default_split(int key_type, bool values, uint64_t max_seg) {
    const Caps c = caps_for(key_type, values);
    SegTuning t;
    uint64_t hi = c.final_cap;
    while (t.classes < (uint32_t)kMaxSegClasses) {
        hi = t.classes + 1 == (uint32_t)kMaxSegClasses ? ~0ull : hi * 4;
        t.upper[t.classes++] = hi;
        if (hi >= max_seg) break;
    }
    return t;
}

int make_seg_geom(int key_type, bool values, uint64_t n, uint64_t S, uint64_t max_seg,
                  const SegTuning &tu, SegGeom &g) {
    g = SegGeom{};
    g.key_type = key_type;
    g.values = values;
    g.n = n;
    g.S = S;
    g.caps = caps_for(key_type, values);
    const Caps &c = g.caps;
    if (n > kMaxItems || tu.classes > (uint32_t)kMaxSegClasses) return DSORT_E_INVALID;
    const uint64_t lim = seg_limit(key_type, values);
    max_seg = clamp_max_seg(n, max_seg, lim);
    if (max_seg > lim) return DSORT_E_UNSUPPORTED;
    g.max_seg = max_seg;
    g.small_cap = c.final_cap;
    const uint32_t ncls = tu.classes ? tu.classes : 1u;
    for (uint32_t k = 0, prev = 0; k < tu.classes; ++k) {  // bounds must increase
        if (tu.upper[k] <= (k ? tu.upper[prev] : (uint64_t)g.small_cap)) return DSORT_E_INVALID;
        prev = k;
    }
    uint64_t lo = g.small_cap;
    for (uint32_t k = 0; k < ncls; ++k) {
        const bool last = k + 1 == ncls;
        uint64_t hi = last ? max_seg : (tu.upper[k] < max_seg ? tu.upper[k] : max_seg);
        uint64_t L = tu.classes && tu.L[k] ? tu.L[k] : c.tile_max;
        uint64_t s = tu.classes ? tu.s[k] : 0;
        if (!seg_L_ok(c, L) || (s && (!is_pow2(s) || s > L || s > kMaxSamples)))
            return DSORT_E_UNSUPPORTED;
        if (hi > lo) {
            uint64_t m = ceil_div(hi, L);
            if (s && (m > kMaxPieces || bucket_bound(m, L, s) > c.final_cap ||
                      m * s > c.samp_cap))
                s = 0;  // cannot bound this call's buckets: this class uses the defaults
            if (!s && !seg_samples(c, m, L)) {
                L = c.tile_max;
                m = ceil_div(hi, L);
            }
            if (!s) s = seg_samples(c, m, L);
            if (!s) return DSORT_E_UNSUPPORTED;
            SegClassGeom &q = g.cls[g.nclasses++];
            q.lo = lo;
            q.hi = hi;
            q.L = (uint32_t)L;
            q.s = (uint32_t)s;
            q.beta = bucket_bound(m, L, s);
            const uint64_t by_size = n / (lo + 1);
            q.gmax = (uint32_t)(S < by_size ? S : by_size);
            q.tiles_max = (uint32_t)(ceil_div(n, L) + q.gmax);
        }
        if (!last) lo = tu.upper[k] > lo ? tu.upper[k] : lo;
        if (lo >= max_seg) break;
    }
    size_t off = 256;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    g.o_status = 0;
    g.o_small_b = take(S * 16);
    g.o_spiece = take(S * 4);
    g.o_slists = take(kNumClasses * S * 4);
    size_t sm = 0, fb = 0;
    for (uint32_t k = 0; k < g.nclasses; ++k) {
        SegClassGeom &q = g.cls[k];
        q.o_tab = take((size_t)q.gmax * 16);
        q.o_tileoff = take(((size_t)q.gmax + 1) * 4);
        sm = std::max(sm, (size_t)q.tiles_max * q.s);
        fb = std::max(fb, (size_t)q.gmax * q.s);
    }
    if (sm) {
        g.o_wkeys = take(n * c.key_bytes);
        if (values) g.o_wvals = take(n * 4);
        g.o_samp = take(sm * c.samp_bytes);
        g.o_samp_sorted = take(sm * c.samp_bytes);
        g.o_counts = take(sm * 4);
        g.o_offs = take(sm * 4);
        g.o_pdst = take(sm * 4);
        g.o_psrc = take(sm * 4);
        g.o_final = take(fb * 16);
        g.o_lists = take(kNumClasses * fb * 4);
    }
    g.total = off;
    return DSORT_OK;
}

size_t seg_workspace_bound(int key_type, bool values, uint64_t n, uint64_t S, uint64_t max_seg) {
    SegGeom g;
    if (make_seg_geom(key_type, values, n, S, max_seg, SegTuning{}, g) != DSORT_OK) return 0;
    size_t ws = g.total;
    const Caps c = caps_for(key_type, values);
    const SegTuning split = seg_default_split(key_type, values, g.max_seg);
    uint32_t Ls[4];
    const int nL = seg_candidate_L(c, Ls);
    // Every trial of the autotuner changes one class to one (L, s) and leaves the others at
    // their defaults; a final choice needs no more than the largest of its trials.
    SegGeom h;
    if (make_seg_geom(key_type, values, n, S, g.max_seg, split, h) == DSORT_OK)
        ws = std::max(ws, h.total);
    uint64_t lo = c.final_cap;
    for (uint32_t k = 0; k < split.classes; ++k) {
        const uint64_t hi = std::min<uint64_t>(split.upper[k], g.max_seg);
        for (int i = 0; i < nL && hi > lo; ++i) {
            const uint64_t s0 = seg_samples(c, ceil_div(hi, Ls[i]), Ls[i]);
            for (uint64_t s = s0; s && s <= 4 * s0; s <<= 1) {
                SegTuning one = split;
                one.L[k] = Ls[i];
                one.s[k] = (uint32_t)s;
                if (make_seg_geom(key_type, values, n, S, g.max_seg, one, h) == DSORT_OK)
                    ws = std::max(ws, h.total);
            }
        }
        lo = split.upper[k];
    }
    return ws;
}

static thread_local char g_last_error[256];

void set_last_error(const char *stage, const char *name, const char *text) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%s)", stage ? stage : "?",
             name ? name : "?", text ? text : "?");
}

}  // namespace dsort

// ---------------------------------------------------------------------------------- C ABI

using dsort::Geom;

static bool plan_ok(const dsort_plan_s *p) { return dsort::plan_valid(p); }

static int geom_for(dsort_plan_s *p, uint64_t n, const Geom **out) {
    if (p->last.n != n || p->last.levels == -2) {
        Geom g;
        int rc = dsort::make_geom(p->key_type, p->values != 0, n, p->tuning, g);
        if (rc != DSORT_OK) return rc;
        p->last = g;
    }
    *out = &p->last;
    return DSORT_OK;
}

// Raises `ws` to the largest workspace any n in [2, max_items] needs under `tu`.  The geometry
// is piecewise in n: on each interval where (levels, rule, s1, s2, sample-sort and scan variants)
// stay fixed, every buffer grows with n, and these pieces never recur once left (the level
// count and the rule only grow with n, and so do s1 and s2 under one rule).  So the largest
// footprint is at the right end of some piece; walk the pieces, finding each right end by
// bisection.
static int workspace_walk(int key_type, bool values, uint64_t max_items, const dsort_tuning_t &tu,
                          size_t &ws) {
    if (max_items < 2) return DSORT_OK;
    auto key = [](const Geom &h) {
        return ((uint64_t)(h.levels + 1) << 56) ^ ((uint64_t)h.plan_rule << 52) ^
               ((uint64_t)h.s1 << 36) ^ ((uint64_t)h.s2 << 12) ^
               ((uint64_t)h.samp_global << 1) ^ (uint64_t)h.scan_large;
    };
    uint64_t lo = 2;
    while (lo <= max_items) {
        Geom h;
        if (dsort::make_geom(key_type, values, lo, tu, h) != DSORT_OK) return DSORT_E_UNSUPPORTED;
        const uint64_t k0 = key(h);
        uint64_t a = lo, b = max_items;
        while (a < b) {
            const uint64_t mid = a + (b - a + 1) / 2;
            Geom t;
            if (dsort::make_geom(key_type, values, mid, tu, t) == DSORT_OK && key(t) == k0)
                a = mid;
            else
                b = mid - 1;
        }
        Geom e;
        dsort::make_geom(key_type, values, a, tu, e);
        if (e.total > ws) ws = e.total;
        lo = a + 1;
    }
    return DSORT_OK;
}

extern "C" {

int dsort_plan(dsort_plan_t *out, int key_type, int with_values, uint64_t max_items,
               uint64_t max_segments, const dsort_tuning_t *tuning, size_t *workspace_bytes) {
    if (!out || !workspace_bytes) return DSORT_E_INVALID;
    *out = nullptr;
    if (key_type != DSORT_U32 && key_type != DSORT_U64 && key_type != DSORT_F32)
        return DSORT_E_INVALID;
    if (with_values != 0 && with_values != 1) return DSORT_E_INVALID;
    if (max_items > dsort::kMaxItems) return DSORT_E_INVALID;
    if (max_segments > dsort::kMaxSegments) return DSORT_E_INVALID;
    dsort_tuning_t tu{};
    if (tuning) tu = *tuning;
    // The workspace must serve every n <= max_items.
    size_t ws = 256;
    int rc = workspace_walk(key_type, with_values != 0, max_items, tu, ws);
    if (rc != DSORT_OK) return rc;
    if (tu.sampling) {
        // a randomized call sorts its oversized buckets by further deterministic runs of the
        // automatic plan, in the same workspace
        rc = workspace_walk(key_type, with_values != 0, max_items, dsort_tuning_t{}, ws);
        if (rc != DSORT_OK) return rc;
    }
    // Segmented calls: every buffer grows with n, S and the longest admissible segment; the
    // bound also covers every tuning the autotuner may choose.
    if (max_segments && max_items) {
        const uint64_t lim = dsort::seg_limit(key_type, with_values != 0);
        const size_t sw = dsort::seg_workspace_bound(key_type, with_values != 0, max_items,
                                                     max_segments,
                                                     max_items < lim ? max_items : lim);
        if (!sw) return DSORT_E_UNSUPPORTED;
        if (sw > ws) ws = sw;
    }
    dsort_plan_s *p = new (std::nothrow) dsort_plan_s{};
    if (!p) return DSORT_E_NOMEM;
    p->magic = dsort::kPlanMagic;
    p->key_type = key_type;
    p->values = with_values;
    p->max_items = max_items;
    p->max_segments = max_segments;
    p->tuning = tu;
    p->workspace = ws;
    p->last.levels = -2;
    *out = p;
    *workspace_bytes = ws;
    return DSORT_OK;
}

int dsort_plan_destroy(dsort_plan_t plan) {
    if (!plan) return DSORT_OK;
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    plan->magic = 0;
    dsort::timing_destroy(plan->timing);
    delete plan;
    return DSORT_OK;
}

const char *dsort_strerror(int status) {
    switch (status) {
        case DSORT_OK: return "success";
        case DSORT_E_INVALID: return "invalid argument";
        case DSORT_E_UNSUPPORTED: return "unsupported request (no feasible level plan)";
        case DSORT_E_NOMEM: return "out of host memory";
        case DSORT_E_HIP: return "HIP runtime error";
        case DSORT_E_CAPACITY: return "request exceeds capacity";
        case DSORT_E_TICKET: return "unknown ticket";
        default: return "unknown status";
    }
}

const char *dsort_last_error(void) { return dsort::g_last_error; }

int dsort_plan_geometry(dsort_plan_t plan, uint64_t n, dsort_geometry_t *out) {
    if (!plan_ok(plan) || !out) return DSORT_E_INVALID;
    if (n > plan->max_items) return DSORT_E_INVALID;
    const Geom *g = nullptr;
    int rc = geom_for(plan, n, &g);
    if (rc != DSORT_OK) return rc;
    memset(out, 0, sizeof(*out));
    out->n = n;
    out->levels = g->levels < 0 ? 0 : (uint32_t)g->levels;
    out->sublist_len = g->L1;
    out->samples = g->s1;
    out->sublists = g->m1;
    out->sublist_len2 = g->L2;
    out->samples2 = g->s2;
    out->max_tiles2 = g->tiles2max;
    out->bucket_capacity = g->caps.final_cap;
    out->bucket_bound = g->beta1;
    out->sample_bytes = g->caps.samp_bytes;
    out->sample_sort_global = g->samp_global ? 1u : 0u;
    out->off_status = g->o_status;
    out->off_samples = g->o_samp;
    out->off_sorted_samples = g->o_samp_sorted;
    out->off_counts = g->o_counts;
    out->off_offsets = g->o_offs;
    out->off_buckets = g->o_buckets1;
    out->workspace_bytes = g->total;
    out->sampling = g->random ? 1u : 0u;
    out->bucket_limit = g->bucket_limit;
    out->off_overflow_count = g->random ? g->o_status + 4ull * dsort::kOverflowWord : 0;
    out->off_overflow_list = g->o_ovf;
    return DSORT_OK;
}

static int sort_common(dsort_plan_t plan, void *d_keys, uint32_t *d_vals, uint64_t n,
                       void *d_ws, void *stream, bool with_values) {
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    if ((plan->values != 0) != with_values) return DSORT_E_INVALID;
    if (n > plan->max_items) return DSORT_E_INVALID;
    if (n <= 1) return DSORT_OK;
    if (!d_keys || !d_ws || (with_values && !d_vals)) return DSORT_E_INVALID;
    if (((uintptr_t)d_ws & 255) != 0) return DSORT_E_INVALID;
    if (((uintptr_t)d_keys & (plan->key_type == DSORT_U64 ? 7 : 3)) != 0) return DSORT_E_INVALID;
    if (with_values && ((uintptr_t)d_vals & 3) != 0) return DSORT_E_INVALID;
    const Geom *g = nullptr;
    int rc = geom_for(plan, n, &g);
    if (rc != DSORT_OK) return rc;
    if (g->total > plan->workspace) return DSORT_E_CAPACITY;
    return dsort::run_pipeline(*g, d_keys, d_vals, d_ws, stream, &plan->timing);
}

int dsort_set_timing(dsort_plan_t plan, int enable) {
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    plan->timing.enabled = enable != 0;
    dsort::timing_reset(plan->timing);
    return DSORT_OK;
}

int dsort_stage_times(dsort_plan_t plan, const char **names, float *avg_ms, uint32_t *launches,
                      int capacity, int *count) {
    if (!plan_ok(plan) || !count || capacity < 0) return DSORT_E_INVALID;
    return dsort::timing_summary(plan->timing, names, avg_ms, launches, capacity, count);
}

static int seg_geom_for(dsort_plan_t plan, uint64_t n, uint64_t S, uint64_t max_segment,
                        dsort::SegGeom &g) {
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    if (n > plan->max_items || S > plan->max_segments) return DSORT_E_INVALID;
    return dsort::make_seg_geom(plan->key_type, plan->values != 0, n, S, max_segment,
                                plan->seg_tuning, g);
}

int dsort_segmented_geometry(dsort_plan_t plan, uint64_t n, uint64_t num_segments,
                             uint64_t max_segment, dsort_seg_geometry_t *out) {
    if (!out) return DSORT_E_INVALID;
    dsort::SegGeom g;
    int rc = seg_geom_for(plan, n, num_segments, max_segment, g);
    if (rc != DSORT_OK) return rc;
    memset(out, 0, sizeof(*out));
    out->n = n;
    out->num_segments = num_segments;
    out->max_segment = g.max_seg;
    out->segment_limit = dsort::seg_limit(plan->key_type, plan->values != 0);
    out->small_capacity = g.small_cap;
    out->classes = g.nclasses;
    for (uint32_t c = 0; c < g.nclasses; ++c) {
        const dsort::SegClassGeom &q = g.cls[c];
        out->class_upper[c] = q.hi;
        out->sublist_len[c] = q.L;
        out->samples[c] = q.s;
        out->max_long_segments[c] = q.gmax;
        out->max_sublists[c] = q.tiles_max;
        out->bucket_bound[c] = q.beta;
    }
    out->off_status = g.o_status;
    out->workspace_bytes = g.total;
    return DSORT_OK;
}

static dsort::SegTuning tuning_from(const dsort_seg_tuning_t &t) {
    dsort::SegTuning s;
    s.classes = t.classes;
    for (int c = 0; c < dsort::kMaxSegClasses; ++c) {
        s.upper[c] = t.upper[c];
        s.L[c] = t.sublist_len[c];
        s.s[c] = t.samples[c];
    }
    return s;
}

static void tuning_to(const dsort::SegTuning &s, dsort_seg_tuning_t &t) {
    memset(&t, 0, sizeof(t));
    t.classes = s.classes;
    for (int c = 0; c < dsort::kMaxSegClasses; ++c) {
        t.upper[c] = s.upper[c];
        t.sublist_len[c] = s.L[c];
        t.samples[c] = s.s[c];
    }
}

extern "C++" {
namespace dsort {
// Checks a tuning against the plan's largest call and installs it.
int plan_set_seg_tuning(dsort_plan_s *plan, const SegTuning &tu) {
    const uint64_t lim = seg_limit(plan->key_type, plan->values != 0);
    SegGeom g;
    const int rc = make_seg_geom(plan->key_type, plan->values != 0, plan->max_items,
                                 plan->max_segments,
                                 plan->max_items < lim ? plan->max_items : lim, tu, g);
    if (rc != DSORT_OK) return rc;
    if (g.total > plan->workspace) return DSORT_E_CAPACITY;
    plan->seg_tuning = tu;
    return DSORT_OK;
}
}  // namespace dsort
}

int dsort_set_seg_tuning(dsort_plan_t plan, const dsort_seg_tuning_t *tuning) {
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    if (!tuning) {
        plan->seg_tuning = dsort::SegTuning{};
        return DSORT_OK;
    }
    if (tuning->classes > (uint32_t)dsort::kMaxSegClasses) return DSORT_E_INVALID;
    if (!plan->max_segments) return DSORT_E_INVALID;
    return dsort::plan_set_seg_tuning(plan, tuning_from(*tuning));
}

int dsort_get_seg_tuning(dsort_plan_t plan, dsort_seg_tuning_t *out) {
    if (!plan_ok(plan) || !out) return DSORT_E_INVALID;
    tuning_to(plan->seg_tuning, *out);
    return DSORT_OK;
}

int dsort_segmented(dsort_plan_t plan, void *d_keys, uint32_t *d_values, uint64_t n,
                    const uint64_t *d_offsets, uint64_t num_segments, uint64_t max_segment,
                    void *d_workspace, void *stream) {
    if (!plan_ok(plan)) return DSORT_E_INVALID;
    if (plan->tuning.sampling) return DSORT_E_UNSUPPORTED;  // randomized samples: plain sorts only
    if ((plan->values != 0) != (d_values != nullptr)) return DSORT_E_INVALID;
    if (n > plan->max_items || num_segments > plan->max_segments) return DSORT_E_INVALID;
    if (n == 0 || num_segments == 0) return DSORT_OK;
    if (!d_keys || !d_offsets || !d_workspace) return DSORT_E_INVALID;
    if (((uintptr_t)d_workspace & 255) != 0 || ((uintptr_t)d_offsets & 7) != 0)
        return DSORT_E_INVALID;
    if (((uintptr_t)d_keys & (plan->key_type == DSORT_U64 ? 7 : 3)) != 0) return DSORT_E_INVALID;
    if (d_values && ((uintptr_t)d_values & 3) != 0) return DSORT_E_INVALID;
    dsort::SegGeom g;
    int rc = seg_geom_for(plan, n, num_segments, max_segment, g);
    if (rc != DSORT_OK) return rc;
    if (g.total > plan->workspace) return DSORT_E_CAPACITY;
    return dsort::run_segmented(g, d_keys, d_values, d_offsets, d_workspace, stream,
                                &plan->timing, 0xFFFFFFFFu, true);
}

int dsort_keys(dsort_plan_t plan, void *d_keys, uint64_t n, void *d_workspace, void *stream) {
    return sort_common(plan, d_keys, nullptr, n, d_workspace, stream, false);
}

int dsort_pairs(dsort_plan_t plan, void *d_keys, uint32_t *d_values, uint64_t n,
                void *d_workspace, void *stream) {
    return sort_common(plan, d_keys, d_values, n, d_workspace, stream, true);
}

}  // extern "C"
