// Autotuner of the segmented sort: per length class of the long segments, the sublist length L
// and the samples per sublist s that sort the caller's batch fastest, measured with HIP events.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "dsort.h"
#include "dsort_internal.h"

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// The current device as the tuning cache names it: architecture, marketing name, CU count.
bool device_id(std::string &out) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    char buf[512];
    snprintf(buf, sizeof(buf), "%s/%s/%dcu", prop.gcnArchName, prop.name,
             prop.multiProcessorCount);
    out = buf;
    return true;
}

void tuning_out(const dsort::SegTuning &t, bool from_cache, dsort_seg_tuning_t *out) {
    if (!out) return;
    memset(out, 0, sizeof(*out));
    out->classes = t.classes;
    out->from_cache = from_cache ? 1u : 0u;
    for (int q = 0; q < dsort::kMaxSegClasses; ++q) {
        out->upper[q] = t.upper[q];
        out->sublist_len[q] = t.L[q];
        out->samples[q] = t.s[q];
    }
}

}  // namespace

extern "C" int dsort_autotune_segmented(dsort_plan_t plan, const void *d_keys,
                                        const uint32_t *d_values, uint64_t n,
                                        const uint64_t *d_offsets, uint64_t num_segments,
                                        uint64_t max_segment, void *d_scratch_keys,
                                        uint32_t *d_scratch_values, void *d_workspace,
                                        void *stream, uint32_t repeats, dsort_seg_tuning_t *out) {
    using namespace dsort;
    if (!plan_valid(plan)) return DSORT_E_INVALID;
    if (plan->tuning.sampling) return DSORT_E_UNSUPPORTED;  // randomized samples: plain sorts only
    const bool vals = plan->values != 0;
    if (vals != (d_values != nullptr) || vals != (d_scratch_values != nullptr))
        return DSORT_E_INVALID;
    if (n > plan->max_items || num_segments > plan->max_segments || num_segments == 0 || n == 0)
        return DSORT_E_INVALID;
    if (!d_keys || !d_offsets || !d_workspace || !d_scratch_keys) return DSORT_E_INVALID;
    if (((uintptr_t)d_workspace & 255) != 0 || ((uintptr_t)d_offsets & 7) != 0)
        return DSORT_E_INVALID;
    const uintptr_t ka = plan->key_type == DSORT_U64 ? 7 : 3;
    if (((uintptr_t)d_keys & ka) || ((uintptr_t)d_scratch_keys & ka)) return DSORT_E_INVALID;
    if (repeats == 0) repeats = 1;
    hipStream_t st = (hipStream_t)stream;
    const Caps c = caps_for(plan->key_type, vals);
    const size_t kbytes = (size_t)n * c.key_bytes;

    SegGeom g0;
    int rc = make_seg_geom(plan->key_type, vals, n, num_segments, max_segment, SegTuning{}, g0);
    if (rc != DSORT_OK) return rc;
    // A result persisted for this device, layout and segment class (DSORT_TUNE_CACHE names the
    // file) is installed without timing, if it still fits this plan.
    const char *cache = getenv("DSORT_TUNE_CACHE");
    if (cache && !*cache) cache = nullptr;
    TuneKey key;
    key.key_type = plan->key_type;
    key.values = vals;
    key.seg_class = tune_seg_class(g0.max_seg);
    if (cache && !device_id(key.device)) cache = nullptr;
    if (cache) {
        SegTuning cached;
        if (tune_cache_lookup(cache, key, cached) &&
            plan_set_seg_tuning(plan, cached) == DSORT_OK) {
            tuning_out(cached, true, out);
            return DSORT_OK;
        }
    }
    SegTuning best = seg_default_split(plan->key_type, vals, g0.max_seg);
    uint32_t Ls[4];
    const int nL = seg_candidate_L(c, Ls);

    Events ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) {
        (void)hipGetLastError();
        return DSORT_E_HIP;
    }
    // One timed run on a fresh copy of the batch: class k of tuning t alone (k >= 0), or the
    // whole batch (k < 0).  The fastest of `repeats` runs counts.
    auto trial = [&](const SegTuning &t, int k, float &ms) -> int {
        SegGeom g;
        int r = make_seg_geom(plan->key_type, vals, n, num_segments, g0.max_seg, t, g);
        if (r != DSORT_OK) return r;
        if (g.total > plan->workspace) return DSORT_E_CAPACITY;
        uint32_t mask = 0xFFFFFFFFu;
        if (k >= 0) {  // the geometry lists only classes with room; find class k among them
            const uint64_t lo = k ? t.upper[k - 1] : c.final_cap;
            uint32_t pos = g.nclasses;
            for (uint32_t q = 0; q < g.nclasses; ++q)
                if (g.cls[q].lo == lo) pos = q;
            if (pos == g.nclasses) return DSORT_E_UNSUPPORTED;
            mask = 1u << pos;
        }
        float bestms = 1e30f;
        for (uint32_t r2 = 0; r2 < repeats; ++r2) {
            if (hipMemcpyAsync(d_scratch_keys, d_keys, kbytes, hipMemcpyDeviceToDevice, st) !=
                    hipSuccess ||
                (vals && hipMemcpyAsync(d_scratch_values, d_values, (size_t)n * 4,
                                        hipMemcpyDeviceToDevice, st) != hipSuccess) ||
                hipEventRecord(ev.a, st) != hipSuccess) {
                (void)hipGetLastError();
                return DSORT_E_HIP;
            }
            r = run_segmented(g, d_scratch_keys, d_scratch_values, d_offsets, d_workspace, st,
                              nullptr, mask, true);
            if (r != DSORT_OK) return r;
            float t_ms = 0.f;
            if (hipEventRecord(ev.b, st) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
                hipEventElapsedTime(&t_ms, ev.a, ev.b) != hipSuccess) {
                (void)hipGetLastError();
                return DSORT_E_HIP;
            }
            bestms = std::min(bestms, t_ms);
        }
        ms = bestms;
        return DSORT_OK;
    };
    auto feasible_skip = [](int r) { return r == DSORT_E_UNSUPPORTED || r == DSORT_E_CAPACITY; };

    // (a) one class for every long segment: each candidate (L, s), whole batch timed
    SegTuning one;
    one.classes = 1;
    one.upper[0] = ~0ull;
    SegTuning best_one = SegTuning{};
    float best_one_ms = 1e30f;
    {
        float ms = 0.f;
        rc = trial(SegTuning{}, -1, ms);
        if (rc != DSORT_OK) return rc;
        best_one_ms = ms;
    }
    for (int i = 0; i < nL && g0.nclasses; ++i) {
        const uint64_t s0 = seg_samples(c, (g0.max_seg + Ls[i] - 1) / Ls[i], Ls[i]);
        for (uint64_t s = s0; s && s <= 4 * s0; s <<= 1) {
            SegTuning t = one;
            t.L[0] = Ls[i];
            t.s[0] = (uint32_t)s;
            float ms = 0.f;
            const int r = trial(t, -1, ms);
            if (feasible_skip(r)) continue;
            if (r != DSORT_OK) return r;
            if (ms < best_one_ms) {
                best_one_ms = ms;
                best_one = t;
            }
        }
    }

    // (b) length classes: each class's candidates timed on that class alone, the others at
    // their defaults; then the whole batch under the combined choice
    uint64_t lo = c.final_cap;
    for (uint32_t k = 0; k < best.classes; ++k) {
        const uint64_t hi = std::min<uint64_t>(best.upper[k], g0.max_seg);
        if (hi <= lo) break;
        float best_ms = 1e30f;
        uint32_t bL = 0, bs = 0;
        for (int i = 0; i < nL; ++i) {
            const uint64_t s0 = seg_samples(c, (hi + Ls[i] - 1) / Ls[i], Ls[i]);
            for (uint64_t s = s0; s && s <= 4 * s0; s <<= 1) {
                SegTuning t = best;
                t.L[k] = Ls[i];
                t.s[k] = (uint32_t)s;
                float ms = 0.f;
                const int r = trial(t, (int)k, ms);
                if (feasible_skip(r)) continue;
                if (r != DSORT_OK) return r;
                if (ms < best_ms) {
                    best_ms = ms;
                    bL = Ls[i];
                    bs = (uint32_t)s;
                }
            }
        }
        best.L[k] = bL;
        best.s[k] = bs;
        lo = best.upper[k];
    }
    if (best.classes > 1) {
        float ms = 0.f;
        const int r = trial(best, -1, ms);
        if (!feasible_skip(r) && r != DSORT_OK) return r;
        if (r != DSORT_OK || ms >= best_one_ms) best = best_one;
    } else {
        best = best_one;
    }
    if (best.classes == 0 && g0.nclasses) {
        // the defaults measured fastest: install them as an explicit tuning, so that the
        // caller sees the (L, s) per class that won
        best.classes = g0.nclasses;
        for (uint32_t q = 0; q < g0.nclasses; ++q) {
            best.upper[q] = q + 1 == g0.nclasses ? ~0ull : g0.cls[q].hi;
            best.L[q] = g0.cls[q].L;
            best.s[q] = g0.cls[q].s;
        }
    }
    rc = plan_set_seg_tuning(plan, best);
    if (rc != DSORT_OK) return rc;
    if (cache) (void)tune_cache_store(cache, key, best);  // a failed write only loses the cache
    tuning_out(best, false, out);
    return DSORT_OK;
}
