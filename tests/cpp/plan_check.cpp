// Host-only checks of the planner (csrc/plan.cpp) built without HIP, plainly and under
// AddressSanitizer/UBSan: the pipeline entry points are replaced by stubs that check what the
// planner hands them.  For many key layouts, sizes and tunings (valid and invalid, Algorithm 1's
// samples and the randomized variant): every call's geometry fits the plan's workspace, every
// intermediate region lies inside it, regions do not overlap, Section 4's bound holds for the
// chosen (L, s), and randomized plans also fit the further deterministic runs they may make.
// Prints "OK <name>" per check group and "ALL OK"; exits non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <utility>
#include <vector>

#include "dsort_internal.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

// ---------------------------------------------------------------- stubs of kernels.hip
static size_t g_calls = 0, g_last_total = 0;
static size_t g_seg_calls = 0;

namespace dsort {
int run_pipeline(const Geom &g, void *, uint32_t *, void *, void *, Timing *) {
    ++g_calls;
    g_last_total = g.total;
    return DSORT_OK;
}
int run_segmented(const SegGeom &g, void *, uint32_t *, const uint64_t *, void *, void *,
                  Timing *, uint32_t, bool) {
    ++g_seg_calls;
    g_last_total = g.total;
    return DSORT_OK;
}
void timing_reset(Timing &t) {
    t.used = 0;
    t.recs.clear();
}
void timing_destroy(Timing &t) {
    t.pool.clear();
    t.recs.clear();
    t.used = 0;
}
int timing_summary(Timing &, const char **, float *, uint32_t *, int, int *count) {
    *count = 0;
    return DSORT_OK;
}
}  // namespace dsort

using dsort::Geom;

// The level-1 regions of a geometry as [offset, offset + bytes) pairs.
static std::vector<std::pair<size_t, size_t>> regions(const Geom &g) {
    std::vector<std::pair<size_t, size_t>> r;
    const size_t sm = (size_t)g.m1 * g.s1, sb = g.caps.samp_bytes;
    auto add = [&](size_t o, size_t b) {
        if (b) r.push_back({o, o + b});
    };
    add(g.o_status, 256);
    add(g.o_wkeys, g.n * g.caps.key_bytes);
    if (g.values) add(g.o_wvals, g.n * 4);
    add(g.o_samp, sm * sb);
    add(g.o_samp_sorted, sm * sb);
    if (g.samp_global) add(g.o_samp_tmp, sm * sb);
    add(g.o_counts, sm * 4);
    add(g.o_offs, sm * 4);
    add(g.o_pdst, sm * 4);
    add(g.o_psrc, sm * 4);
    add(g.o_partial, (size_t)g.scan_nrb * g.s1 * 4);
    add(g.o_buckets1, (size_t)g.s1 * 16);
    if (g.levels == 2) {
        const size_t sm2 = (size_t)g.tiles2max * g.s2;
        add(g.o_tileoff2, ((size_t)g.s1 + 1) * 4);
        add(g.o_samp2, sm2 * sb);
        add(g.o_samp2_sorted, sm2 * sb);
        add(g.o_counts2, sm2 * 4);
        add(g.o_offs2, sm2 * 4);
        add(g.o_pdst2, sm2 * 4);
        add(g.o_psrc2, sm2 * 4);
        add(g.o_final, (size_t)g.final_buckets * 16);
    }
    add(g.o_lists, (size_t)8 * g.final_buckets * 4);
    if (g.random) add(g.o_ovf, (size_t)g.s1 * 4);
    return r;
}

static void check_geom(const Geom &g) {
    if (g.levels <= 0) {
        CHECK(g.total >= 256);
        return;
    }
    auto r = regions(g);
    std::sort(r.begin(), r.end());
    for (size_t i = 0; i < r.size(); ++i) {
        CHECK(r[i].second <= g.total);
        CHECK(r[i].first % 256 == 0);
        if (i) CHECK(r[i - 1].second <= r[i].first);  // disjoint
    }
    const uint64_t m = g.m1, L = g.L1, s = g.s1;
    CHECK(m == (g.n + L - 1) / L);
    CHECK(L % s == 0);
    CHECK(g.beta1 == 2 * m * L / s - m);  // Section 4's bound, exact form
    if (g.levels == 1) {
        CHECK(g.beta1 <= g.caps.final_cap);
        CHECK(m <= 256);
    } else {
        CHECK(g.m2max <= 256);
        CHECK((uint64_t)g.m2max * g.L2 >= g.beta1);
        CHECK((uint64_t)g.m2max * (2 * g.L2 / g.s2 - 1) <= g.caps.final_cap);
        CHECK((uint64_t)g.m2max * g.s2 <= g.caps.samp_cap);
        CHECK(g.tiles2max == (g.n + g.L2 - 1) / g.L2 + s);
    }
    if (g.random) {
        if (g.levels == 1)
            CHECK(g.bucket_limit == g.caps.final_cap);
        else
            CHECK(g.bucket_limit >= g.beta1 && g.bucket_limit % g.L2 == 0);
    } else {
        CHECK(g.bucket_limit == 0);
    }
}

static void plan_sizes(int kt, int vals, uint64_t max_items, const dsort_tuning_t *tu,
                       std::mt19937_64 &rng) {
    dsort_plan_t p = nullptr;
    size_t ws = 0;
    const int rc = dsort_plan(&p, kt, vals, max_items, 0, tu, &ws);
    if (rc != DSORT_OK) {
        CHECK(rc == DSORT_E_UNSUPPORTED || rc == DSORT_E_INVALID);
        CHECK(p == nullptr);
        return;
    }
    std::vector<uint64_t> ns = {0, 1, 2, 3, max_items, max_items - 1, max_items / 2};
    for (int i = 0; i < 40; ++i) ns.push_back(rng() % (max_items + 1));
    for (uint64_t sh = 1; sh <= max_items; sh <<= 1) ns.push_back(sh);
    for (uint64_t n : ns) {
        if (n > max_items) continue;
        dsort_geometry_t out;
        CHECK(dsort_plan_geometry(p, n, &out) == DSORT_OK);
        CHECK(out.workspace_bytes <= ws);
        Geom g;
        dsort_tuning_t t{};
        if (tu) t = *tu;
        CHECK(dsort::make_geom(kt, vals != 0, n, t, g) == DSORT_OK);
        CHECK(g.total == out.workspace_bytes);
        check_geom(g);
        if (g.random) {  // further runs use the automatic plan in the same workspace
            for (uint64_t part : {n, n / 2, n / 3 + 1}) {
                Geom h;
                CHECK(dsort::make_geom(kt, vals != 0, part, dsort_tuning_t{}, h) == DSORT_OK);
                CHECK(h.total <= ws);
            }
        }
        // a sorting call hands the same geometry to the pipeline
        const size_t before = g_calls;
        void *fake = (void *)0x100000;
        const int r2 = vals ? dsort_pairs(p, fake, (uint32_t *)fake, n, fake, nullptr)
                            : dsort_keys(p, fake, n, fake, nullptr);
        CHECK(r2 == DSORT_OK);
        if (n >= 2) {
            CHECK(g_calls == before + 1);
            CHECK(g_last_total <= ws);
        } else {
            CHECK(g_calls == before);
        }
    }
    CHECK(dsort_plan_destroy(p) == DSORT_OK);
}

static void check_plans() {
    std::mt19937_64 rng(12345);
    const int kts[3] = {DSORT_U32, DSORT_U64, DSORT_F32};
    for (int kt : kts)
        for (int vals = 0; vals < 2; ++vals)
            for (uint64_t mx : {2ull, 100ull, 32768ull, 32769ull, 70001ull, 4194304ull,
                                 (1ull << 24) + 3, (1ull << 27) + 5})
                for (int sampling = 0; sampling < 2; ++sampling) {
                    dsort_tuning_t t{};
                    t.sampling = (uint32_t)sampling;
                    t.seed = rng();
                    plan_sizes(kt, vals, mx, &t, rng);
                }
    printf("OK automatic plans\n");
    // tunings, feasible and not
    for (int i = 0; i < 300; ++i) {
        dsort_tuning_t t{};
        t.sublist_len = 1u << (rng() % 16);
        t.samples = rng() % 3 ? 1u << (rng() % 11) : 0;
        t.sublist_len2 = rng() % 2 ? 1u << (rng() % 16) : 0;
        t.samples2 = rng() % 3 ? 1u << (rng() % 10) : 0;
        t.levels = (uint32_t)(rng() % 3);
        t.sampling = (uint32_t)(rng() % 2);
        t.seed = rng();
        const int kt = kts[rng() % 3];
        const uint64_t mx = 2 + rng() % (1u << (10 + rng() % 16));
        plan_sizes(kt, (int)(rng() % 2), mx, &t, rng);
    }
    printf("OK tuned plans\n");
    // the largest plans of each layout
    plan_sizes(DSORT_U32, 0, 1108377600ull, nullptr, rng);
    plan_sizes(DSORT_U64, 1, 286326784ull, nullptr, rng);
    dsort_plan_t p = nullptr;
    size_t ws = 0;
    CHECK(dsort_plan(&p, DSORT_U32, 0, 1108377601ull, 0, nullptr, &ws) == DSORT_E_UNSUPPORTED);
    CHECK(dsort_plan(&p, DSORT_U64, 1, 286326785ull, 0, nullptr, &ws) == DSORT_E_UNSUPPORTED);
    printf("OK size limits\n");
}

static void check_segmented() {
    std::mt19937_64 rng(777);
    const int kts[3] = {DSORT_U32, DSORT_U64, DSORT_F32};
    for (int i = 0; i < 200; ++i) {
        const int kt = kts[rng() % 3], vals = (int)(rng() % 2);
        const uint64_t n = 1 + rng() % (1u << (8 + rng() % 20));
        const uint64_t S = 1 + rng() % 5000;
        dsort_plan_t p = nullptr;
        size_t ws = 0;
        CHECK(dsort_plan(&p, kt, vals, n, S, nullptr, &ws) == DSORT_OK);
        for (int j = 0; j < 10; ++j) {
            const uint64_t nn = rng() % (n + 1), SS = 1 + rng() % S;
            const uint64_t ms = rng() % 2 ? 0 : rng() % (nn + 1);
            dsort_seg_geometry_t out;
            const int rc = dsort_segmented_geometry(p, nn, SS, ms, &out);
            CHECK(rc == DSORT_OK || rc == DSORT_E_UNSUPPORTED);
            if (rc == DSORT_OK) CHECK(out.workspace_bytes <= ws);
            dsort_seg_tuning_t t{};
            t.classes = (uint32_t)(rng() % 5);
            uint64_t up = out.small_capacity ? out.small_capacity : 1;
            for (uint32_t c = 0; c < t.classes; ++c) {
                up += 1 + rng() % (up * 8);
                t.upper[c] = up;
                t.sublist_len[c] = rng() % 2 ? 1u << (8 + rng() % 7) : 0;
                t.samples[c] = rng() % 2 ? 1u << (rng() % 10) : 0;
            }
            const int rs = dsort_set_seg_tuning(p, &t);
            CHECK(rs == DSORT_OK || rs == DSORT_E_UNSUPPORTED || rs == DSORT_E_CAPACITY ||
                  rs == DSORT_E_INVALID);
            if (dsort_segmented_geometry(p, nn, SS, ms, &out) == DSORT_OK)
                CHECK(out.workspace_bytes <= ws);
            void *fake = (void *)0x100000;
            const int r3 = dsort_segmented(p, fake, vals ? (uint32_t *)fake : nullptr, nn,
                                           (const uint64_t *)fake, SS, ms, fake, nullptr);
            CHECK(r3 == DSORT_OK || r3 == DSORT_E_UNSUPPORTED);
            if (r3 == DSORT_OK && nn) CHECK(g_last_total <= ws);
            CHECK(dsort_set_seg_tuning(p, nullptr) == DSORT_OK);
        }
        CHECK(dsort_plan_destroy(p) == DSORT_OK);
    }
    printf("OK segmented geometries\n");
}

static void check_errors() {
    dsort_plan_t p = nullptr;
    size_t ws = 0;
    CHECK(dsort_plan(nullptr, DSORT_U32, 0, 10, 0, nullptr, &ws) == DSORT_E_INVALID);
    CHECK(dsort_plan(&p, 0, 0, 10, 0, nullptr, &ws) == DSORT_E_INVALID);
    CHECK(dsort_plan(&p, DSORT_U32, 0, 1ull << 33, 0, nullptr, &ws) == DSORT_E_INVALID);
    dsort_tuning_t t{};
    t.sampling = 2;
    CHECK(dsort_plan(&p, DSORT_U32, 0, 1000, 0, &t, &ws) == DSORT_E_UNSUPPORTED);
    CHECK(dsort_plan(&p, DSORT_U32, 0, 1000, 0, nullptr, &ws) == DSORT_OK);
    void *fake = (void *)0x100000;
    CHECK(dsort_keys(p, nullptr, 500, fake, nullptr) == DSORT_E_INVALID);
    CHECK(dsort_keys(p, fake, 1001, fake, nullptr) == DSORT_E_INVALID);
    CHECK(dsort_keys(p, (void *)0x100002, 500, fake, nullptr) == DSORT_E_INVALID);
    CHECK(dsort_pairs(p, fake, (uint32_t *)fake, 500, fake, nullptr) == DSORT_E_INVALID);
    CHECK(dsort_plan_geometry(p, 1001, nullptr) == DSORT_E_INVALID);
    CHECK(dsort_plan_destroy(p) == DSORT_OK);
    CHECK(dsort_plan_destroy(nullptr) == DSORT_OK);
    CHECK(strlen(dsort_strerror(-4)) > 0);
    printf("OK errors\n");
}

int main() {
    check_errors();
    check_plans();
    check_segmented();
    printf("ALL OK\n");
    return 0;
}
