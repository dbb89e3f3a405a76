/* Runs the oracle (oracle/dss_oracle.c) built plainly and under AddressSanitizer/UBSan over
 * many small random inputs: every key type, with and without values, both sampling modes,
 * sizes that pad the last sublist, and (L, s) from 1 to the whole input.  Each run's output
 * must equal the oracle's stable sort, and its trace must satisfy Algorithm 1's bookkeeping
 * (row sums L, bucket-major offsets ending at n', buckets in Section 4's bound for chunk-end
 * samples).  Prints "ALL OK"; exits non-zero on the first failure. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t *sample_key, *sample_pos, *splitter_key, *splitter_pos, *count, *offset,
        *bucket_size, *reloc_key;
    uint32_t *reloc_val;
} trace_t;

int oracle_dss_sampled(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n,
                       uint64_t L, uint64_t s, int sampling, uint64_t seed, void *keys_out,
                       uint32_t *vals_out, trace_t *tr);
int oracle_stable_sort(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n,
                       void *keys_out, uint32_t *vals_out);

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);           \
            exit(1);                                                               \
        }                                                                          \
    } while (0)

static uint64_t rng_state = 88172645463325252ull;
static uint64_t rnd(void) { /* xorshift64 */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

int main(void) {
    long runs = 0;
    for (int iter = 0; iter < 3000; ++iter) {
        const int kind = 1 + (int)(rnd() % 3);
        const size_t kb = kind == 2 ? 8 : 4;
        const uint64_t n = rnd() % 300;
        const uint64_t L = 1ull << (rnd() % 9);
        const uint64_t s = 1ull << (rnd() % 9);
        if (s > L) continue;
        const int sampling = (int)(rnd() % 2);
        const int with_vals = (int)(rnd() % 2);
        const uint64_t distinct = 1 + rnd() % 40;
        void *keys = malloc(n * kb + 8), *out = malloc(n * kb + 8), *want = malloc(n * kb + 8);
        uint32_t *vals = malloc(n * 4 + 4), *ov = malloc(n * 4 + 4), *wv = malloc(n * 4 + 4);
        for (uint64_t t = 0; t < n; ++t) {
            const uint64_t r = rnd();
            if (kind == 2) ((uint64_t *)keys)[t] = r % 4 == 0 ? ~0ull : (r >> 8) % distinct;
            else ((uint32_t *)keys)[t] = r % 4 == 0 ? 0xFFFFFFFFu : (uint32_t)((r >> 8) % distinct);
            vals[t] = (uint32_t)t;
        }
        const uint64_t m = n ? (n + L - 1) / L : 0, np = m * L;
        trace_t tr;
        tr.sample_key = malloc((m * s + 1) * 8);
        tr.sample_pos = malloc((m * s + 1) * 8);
        tr.splitter_key = malloc((s + 1) * 8);
        tr.splitter_pos = malloc((s + 1) * 8);
        tr.count = malloc((m * s + 1) * 8);
        tr.offset = malloc((m * s + 1) * 8);
        tr.bucket_size = malloc((s + 1) * 8);
        tr.reloc_key = malloc((np + 1) * 8);
        tr.reloc_val = malloc((np + 1) * 4);
        CHECK(oracle_dss_sampled(kind, keys, with_vals ? vals : NULL, n, L, s, sampling,
                                 rnd(), out, with_vals ? ov : NULL, &tr) == 0);
        CHECK(oracle_stable_sort(kind, keys, with_vals ? vals : NULL, n, want,
                                 with_vals ? wv : NULL) == 0);
        CHECK(memcmp(out, want, n * kb) == 0);
        if (with_vals) CHECK(memcmp(ov, wv, n * 4) == 0);
        if (n) {
            uint64_t run = 0;
            for (uint64_t j = 0; j < s; ++j) {
                uint64_t col = 0;
                for (uint64_t i = 0; i < m; ++i) {
                    CHECK(tr.offset[i * s + j] == run);
                    run += tr.count[i * s + j];
                    col += tr.count[i * s + j];
                }
                CHECK(col == tr.bucket_size[j]);
                if (!sampling) {
                    CHECK(tr.bucket_size[j] >= m);
                    CHECK(tr.bucket_size[j] <= 2 * np / s - m);
                }
            }
            CHECK(run == np);
            for (uint64_t i = 0; i < m; ++i) {
                uint64_t row = 0;
                for (uint64_t j = 0; j < s; ++j) row += tr.count[i * s + j];
                CHECK(row == L);
            }
            for (uint64_t q = 1; q < m * s; ++q)
                CHECK(tr.sample_key[q - 1] < tr.sample_key[q] ||
                      (tr.sample_key[q - 1] == tr.sample_key[q] &&
                       tr.sample_pos[q - 1] <= tr.sample_pos[q]));
        }
        free(keys); free(out); free(want); free(vals); free(ov); free(wv);
        free(tr.sample_key); free(tr.sample_pos); free(tr.splitter_key); free(tr.splitter_pos);
        free(tr.count); free(tr.offset); free(tr.bucket_size); free(tr.reloc_key);
        free(tr.reloc_val);
        ++runs;
    }
    printf("%ld runs\nALL OK\n", runs);
    return 0;
}
