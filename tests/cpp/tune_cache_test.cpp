// Host-only test of the persisted autotuner results (csrc/tune_cache.cpp): round trips, keys
// that differ in one field, replacement in place, foreign lines kept, a missing file, an
// unwritable path.  Prints "ALL OK"; exits non-zero on the first failure.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <string>

#include "dsort_internal.h"

using namespace dsort;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

static SegTuning make(uint32_t seed) {
    SegTuning t;
    t.classes = 1 + seed % 4;
    for (uint32_t q = 0; q < t.classes; ++q) {
        t.upper[q] = q + 1 == t.classes ? ~0ull : 32768ull << (2 * q + seed % 3);
        t.L[q] = 1u << (10 + (seed + q) % 5);
        t.s[q] = 1u << ((seed * 7 + q) % 9);
    }
    return t;
}

static bool same(const SegTuning &a, const SegTuning &b) {
    if (a.classes != b.classes) return false;
    for (int q = 0; q < kMaxSegClasses; ++q)
        if (a.upper[q] != b.upper[q] || a.L[q] != b.L[q] || a.s[q] != b.s[q]) return false;
    return true;
}

int main(int argc, char **argv) {
    const std::string dir = argc > 1 ? argv[1] : "/tmp";
    const std::string path = dir + "/tune_cache_test.txt";
    remove(path.c_str());
    TuneKey k;
    k.device = "gfx950/AMD Instinct MI355X/256cu";
    k.key_type = DSORT_F32;
    k.values = false;
    k.seg_class = 20;
    SegTuning out;
    CHECK(!tune_cache_lookup(path.c_str(), k, out));  // no file yet
    CHECK(tune_seg_class(1) == 0 && tune_seg_class(2) == 1 && tune_seg_class(1048576) == 20 &&
          tune_seg_class(1048577) == 21);
    const SegTuning a = make(3), b = make(6), c = make(11);
    CHECK(tune_cache_store(path.c_str(), k, a));
    CHECK(tune_cache_lookup(path.c_str(), k, out) && same(out, a));
    TuneKey k2 = k;
    k2.values = true;
    CHECK(!tune_cache_lookup(path.c_str(), k2, out));
    CHECK(tune_cache_store(path.c_str(), k2, b));
    TuneKey k3 = k;
    k3.seg_class = 19;
    TuneKey k4 = k;
    k4.device = "gfx942/other device/304cu";
    CHECK(!tune_cache_lookup(path.c_str(), k3, out) && !tune_cache_lookup(path.c_str(), k4, out));
    CHECK(tune_cache_lookup(path.c_str(), k, out) && same(out, a));
    CHECK(tune_cache_lookup(path.c_str(), k2, out) && same(out, b));
    // a foreign line survives a store; replacing a key keeps one line for it
    {
        FILE *f = fopen(path.c_str(), "a");
        CHECK(f);
        fprintf(f, "not a tuning line\n");
        fclose(f);
    }
    CHECK(tune_cache_store(path.c_str(), k, c));
    CHECK(tune_cache_lookup(path.c_str(), k, out) && same(out, c));
    int lines = 0, foreign = 0;
    {
        FILE *f = fopen(path.c_str(), "r");
        char buf[1024];
        while (fgets(buf, sizeof(buf), f)) {
            ++lines;
            foreign += strstr(buf, "not a tuning line") != nullptr;
        }
        fclose(f);
    }
    CHECK(lines == 3 && foreign == 1);
    // spaces in a device name do not split the key
    TuneKey k5 = k;
    k5.device = "gfx950/AMD Instinct MI355X OAM/256cu";
    CHECK(tune_cache_store(path.c_str(), k5, b));
    CHECK(tune_cache_lookup(path.c_str(), k5, out) && same(out, b));
    CHECK(tune_cache_lookup(path.c_str(), k, out) && same(out, c));
    // an unwritable location fails cleanly
    CHECK(!tune_cache_store("/nonexistent-dir/x/tune.txt", k, a));
    CHECK(!tune_cache_lookup(nullptr, k, out) && !tune_cache_store(nullptr, k, a));
    remove(path.c_str());
    printf("ALL OK\n");
    return 0;
}
