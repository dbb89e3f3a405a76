/*
 * Oracle: plain single-threaded deterministic sample sort ("GPU Bucket Sort", Algorithm 1 of
 * Dehne & Zaboli, "Deterministic Sample Sort For GPUs", Section 4).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load this library.  It shares no code, header, table or helper with the HIP path.
 *
 * The method's result has a plain definition: the keys in non-decreasing key order, and for
 * key/value input the stable sort by key (equal keys keep input order).  This file does not
 * shortcut to that definition: it walks the nine steps of Algorithm 1 in the paper's order and
 * notation so that every intermediate (samples, global samples, bucket sizes a_ij, start
 * positions l_ij, relocated array) can be compared with the GPU pipeline at the same (L, s).
 * Library routines used as steps: qsort (every sort below orders items that are pairwise
 * distinct under the comparator, so qsort's lack of stability cannot change the result).
 *
 * Readings of points the paper leaves open (each also listed in the design notes):
 *  R1  "equidistant samples" of a sorted sublist of L = n/m items are the items at sorted
 *      positions k*w - 1 (0-based), k = 1..s, with w = L/s (the last item of each chunk).
 *  R2  the s "global samples" (splitters) are S[j*m - 1], j = 1..s, of the sorted sample list
 *      S; bucket j holds the items in (g_{j-1}, g_j] with g_0 = -infinity; g_s is the global
 *      maximum, so there are exactly s buckets.
 *  R3  items are compared under the strict total order (key, sublist i, sorted rank r); a
 *      sample is the composite (key, i*L + r).  Without this tie-break the bucket bound of
 *      Section 4 fails for repeated keys.
 *  R4  n need not be a multiple of L: the last sublist is padded with items whose key is the
 *      type's maximum; under R3 they sort after every real item and are dropped at the end.
 *  R5  float32 keys are ordered by the IEEE 754 totalOrder image of their bit pattern.
 *  R8  the randomized-splitter variant (the comparison method of Sections 1 and 3, whose
 *      buckets come from randomly selected items): Step 3 takes the items at s random sorted
 *      positions of each sublist instead of the chunk ends.  Sample k (0-based) of sublist i
 *      (0-based) sits at position ((d >> 32) * L) >> 32, where d is draw i*s + k of the
 *      SplitMix64 stream of `seed` (draw c is mix(seed + (c + 1) * 0x9E3779B97F4A7C15), mix
 *      the generator's published finaliser); positions may repeat.  A random sample need not
 *      be the maximum, so the last bucket is closed by +infinity instead of S[sm - 1]: bucket s
 *      takes every item above g_{s-1}.  Every other step is unchanged; the bucket bound of
 *      Section 4 no longer holds for this variant.
 *
 * Parity status: every function here is pinned by the CPU tests (insertion sort and exhaustive
 * small inputs, numpy's stable argsort, the bucket bound, closed forms for sorted and all-equal
 * input, a hand-worked example).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_U32 1
#define ORACLE_U64 2
#define ORACLE_F32 3

#define ORACLE_OK 0
#define ORACLE_E_INVALID (-1)
#define ORACLE_E_NOMEM (-3)

typedef struct {
    uint64_t key; /* order key: the u32/u64 value, or the f32 totalOrder image */
    uint64_t idx; /* input index; pads get n, n+1, ... (R4) */
    uint32_t val;
} item_t;

typedef struct {
    uint64_t key; /* key of the sampled item */
    uint64_t pos; /* i*L + r: sublist and sorted rank of the sampled item (R3) */
} sample_t;

/* Every output pointer may be NULL.  Sizes: m = ceil(n/L). */
typedef struct {
    uint64_t *sample_key;   /* m*s, sorted (Step 4) */
    uint64_t *sample_pos;   /* m*s */
    uint64_t *splitter_key; /* s (Step 5) */
    uint64_t *splitter_pos; /* s */
    uint64_t *count;        /* m*s, row i holds a_i1..a_is (Step 6) */
    uint64_t *offset;       /* m*s, row i holds l_i1..l_is (Step 7) */
    uint64_t *bucket_size;  /* s, |B_j| */
    uint64_t *reloc_key;    /* m*L: keys after Step 8 (pads included), in key-type bits */
    uint32_t *reloc_val;    /* m*L */
} oracle_trace_t;

/* ---------------------------------------------------------------- key order (R5) */

/* totalOrder image of a binary32 pattern: negative patterns are complemented, positive ones
 * get the sign bit set, so unsigned order of the image is IEEE totalOrder. */
uint32_t oracle_f32_order(uint32_t bits) {
    return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}

uint32_t oracle_f32_unorder(uint32_t image) {
    return (image & 0x80000000u) ? (image & 0x7FFFFFFFu) : ~image;
}

static uint64_t key_of(int kind, const void *keys, uint64_t t) {
    if (kind == ORACLE_U64) return ((const uint64_t *)keys)[t];
    uint32_t b = ((const uint32_t *)keys)[t];
    return kind == ORACLE_F32 ? (uint64_t)oracle_f32_order(b) : (uint64_t)b;
}

static void store_key(int kind, void *keys, uint64_t t, uint64_t key) {
    if (kind == ORACLE_U64) {
        ((uint64_t *)keys)[t] = key;
    } else {
        uint32_t k = (uint32_t)key;
        ((uint32_t *)keys)[t] = kind == ORACLE_F32 ? oracle_f32_unorder(k) : k;
    }
}

static uint64_t key_max(int kind) { return kind == ORACLE_U64 ? UINT64_MAX : (uint64_t)UINT32_MAX; }

/* ---------------------------------------------------------------- comparators */

/* Items of one sublist or one bucket: (key, input index) is the stable key order. */
static int cmp_item(const void *pa, const void *pb) {
    const item_t *a = (const item_t *)pa, *b = (const item_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Samples: lexicographic (key, i*L + r), R3. */
static int cmp_sample(const void *pa, const void *pb) {
    const sample_t *a = (const sample_t *)pa, *b = (const sample_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
    return 0;
}

/* (key, pos) <= (gkey, gpos) in the order of R3. */
static int composite_le(uint64_t key, uint64_t pos, uint64_t gkey, uint64_t gpos) {
    return key < gkey || (key == gkey && pos <= gpos);
}

/* ---------------------------------------------------------------- the definition */

/* The plain definition of the result: stable sort by key order (one qsort over distinct
 * (key, input index) pairs).  vals_in/vals_out may be NULL. */
int oracle_stable_sort(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n,
                       void *keys_out, uint32_t *vals_out) {
    if (kind < ORACLE_U32 || kind > ORACLE_F32) return ORACLE_E_INVALID;
    if (n == 0) return ORACLE_OK;
    item_t *it = (item_t *)malloc(n * sizeof(item_t));
    if (!it) return ORACLE_E_NOMEM;
    for (uint64_t t = 0; t < n; ++t) {
        it[t].key = key_of(kind, keys_in, t);
        it[t].idx = t;
        it[t].val = vals_in ? vals_in[t] : 0;
    }
    qsort(it, n, sizeof(item_t), cmp_item);
    for (uint64_t t = 0; t < n; ++t) {
        store_key(kind, keys_out, t, it[t].key);
        if (vals_out) vals_out[t] = it[t].val;
    }
    free(it);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- random positions (R8) */

/* Draw c of the SplitMix64 stream seeded with `seed` (Steele, Lea and Flood 2014): the state
 * after c + 1 steps of adding the golden-ratio increment, passed through the finaliser. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Sorted position (in [0, L)) of random sample k of sublist i (R8). */
static uint64_t random_position(uint64_t seed, uint64_t i, uint64_t k, uint64_t s, uint64_t L) {
    const uint64_t d = oracle_splitmix64(seed, i * s + k);
    return ((d >> 32) * L) >> 32;
}

/* ---------------------------------------------------------------- Algorithm 1 */

int oracle_dss_sampled(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n,
                       uint64_t L, uint64_t s, int sampling, uint64_t seed, void *keys_out,
                       uint32_t *vals_out, oracle_trace_t *tr);

/* Runs Algorithm 1 with sublist length L (= n/m) and s samples per sublist.
 * Requires L >= 1, 1 <= s <= L and s dividing L.  vals_in/vals_out/tr may be NULL. */
int oracle_dss(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n, uint64_t L,
               uint64_t s, void *keys_out, uint32_t *vals_out, oracle_trace_t *tr) {
    return oracle_dss_sampled(kind, keys_in, vals_in, n, L, s, 0, 0, keys_out, vals_out, tr);
}

/* Algorithm 1 with the samples of Step 3 taken at the chunk ends (sampling = 0, R1) or at
 * random positions drawn from `seed` (sampling = 1, R8, L < 2^32). */
int oracle_dss_sampled(int kind, const void *keys_in, const uint32_t *vals_in, uint64_t n,
                       uint64_t L, uint64_t s, int sampling, uint64_t seed, void *keys_out,
                       uint32_t *vals_out, oracle_trace_t *tr) {
    if (kind < ORACLE_U32 || kind > ORACLE_F32) return ORACLE_E_INVALID;
    if (L == 0 || s == 0 || s > L || L % s != 0) return ORACLE_E_INVALID;
    if (sampling != 0 && (sampling != 1 || L >= (1ull << 32))) return ORACLE_E_INVALID;
    if (n == 0) return ORACLE_OK;

    /* Step 1: split A into m sublists of L items (R4: pad the last one). */
    const uint64_t m = (n + L - 1) / L;
    const uint64_t np = m * L;
    const uint64_t w = L / s;
    item_t *A = (item_t *)malloc(np * sizeof(item_t));       /* sublist i = A[i*L .. i*L+L) */
    item_t *out = (item_t *)malloc(np * sizeof(item_t));     /* Step 8 target */
    sample_t *S = (sample_t *)malloc(m * s * sizeof(sample_t));
    sample_t *g = (sample_t *)malloc(s * sizeof(sample_t));
    uint64_t *r = (uint64_t *)malloc(m * (s + 1) * sizeof(uint64_t)); /* r[i][j], j = 0..s */
    uint64_t *a = (uint64_t *)malloc(m * s * sizeof(uint64_t));
    uint64_t *l = (uint64_t *)malloc(m * s * sizeof(uint64_t));
    uint64_t *bsz = (uint64_t *)malloc(s * sizeof(uint64_t));
    if (!A || !out || !S || !g || !r || !a || !l || !bsz) {
        free(A); free(out); free(S); free(g); free(r); free(a); free(l); free(bsz);
        return ORACLE_E_NOMEM;
    }
    for (uint64_t t = 0; t < np; ++t) {
        if (t < n) {
            A[t].key = key_of(kind, keys_in, t);
            A[t].val = vals_in ? vals_in[t] : 0;
        } else {
            A[t].key = key_max(kind);
            A[t].val = 0;
        }
        A[t].idx = t;
    }

    /* Step 2: sort every sublist locally (stable: ties keep input order). */
    for (uint64_t i = 0; i < m; ++i) qsort(A + i * L, L, sizeof(item_t), cmp_item);

    /* Step 3: s equidistant samples per sorted sublist (R1), or s random ones (R8), as
     * composites (R3). */
    for (uint64_t i = 0; i < m; ++i)
        for (uint64_t k = 1; k <= s; ++k) {
            uint64_t rk = sampling ? random_position(seed, i, k - 1, s, L) : k * w - 1;
            S[i * s + (k - 1)].key = A[i * L + rk].key;
            S[i * s + (k - 1)].pos = i * L + rk;
        }

    /* Step 4: sort all sm samples. */
    qsort(S, m * s, sizeof(sample_t), cmp_sample);

    /* Step 5: s equidistant global samples (R2). */
    for (uint64_t j = 1; j <= s; ++j) g[j - 1] = S[j * m - 1];

    /* Step 6: locate every global sample in every sorted sublist.  r_ij is the number of items
     * (A_i[x], i, x) that are <= g_j; the predicate holds on a prefix of the sorted sublist,
     * so it is found by bisection on x.  a_ij = r_ij - r_i,j-1 with r_i0 = 0. */
    for (uint64_t i = 0; i < m; ++i) {
        r[i * (s + 1)] = 0;
        for (uint64_t j = 1; j <= s; ++j) {
            uint64_t lo = 0, hi = L; /* invariant: pred(x) for x < lo, !pred(x) for x >= hi */
            if (sampling && j == s) lo = L; /* R8: the last bucket is closed by +infinity */
            while (lo < hi) {
                uint64_t x = lo + (hi - lo) / 2;
                if (composite_le(A[i * L + x].key, i * L + x, g[j - 1].key, g[j - 1].pos))
                    lo = x + 1;
                else
                    hi = x;
            }
            r[i * (s + 1) + j] = lo;
            a[i * s + (j - 1)] = lo - r[i * (s + 1) + j - 1];
        }
    }

    /* Step 7: exclusive prefix sum over a_11..a_m1, a_12..a_m2, ..., a_1s..a_ms. */
    uint64_t run = 0;
    for (uint64_t j = 0; j < s; ++j) {
        bsz[j] = 0;
        for (uint64_t i = 0; i < m; ++i) {
            l[i * s + j] = run;
            run += a[i * s + j];
            bsz[j] += a[i * s + j];
        }
    }

    /* Step 8: move every A_ij to l_ij; bucket B_j = A_1j u ... u A_mj. */
    for (uint64_t i = 0; i < m; ++i)
        for (uint64_t j = 0; j < s; ++j)
            for (uint64_t x = 0; x < a[i * s + j]; ++x)
                out[l[i * s + j] + x] = A[i * L + r[i * (s + 1) + j] + x];

    if (tr) {
        for (uint64_t q = 0; q < m * s; ++q) {
            if (tr->sample_key) tr->sample_key[q] = S[q].key;
            if (tr->sample_pos) tr->sample_pos[q] = S[q].pos;
            if (tr->count) tr->count[q] = a[q];
            if (tr->offset) tr->offset[q] = l[q];
        }
        for (uint64_t j = 0; j < s; ++j) {
            if (tr->splitter_key) tr->splitter_key[j] = g[j].key;
            if (tr->splitter_pos) tr->splitter_pos[j] = g[j].pos;
            if (tr->bucket_size) tr->bucket_size[j] = bsz[j];
        }
        for (uint64_t t = 0; t < np; ++t) {
            if (tr->reloc_key) store_key(kind, tr->reloc_key, t, out[t].key);
            if (tr->reloc_val) tr->reloc_val[t] = out[t].val;
        }
    }

    /* Step 9: sort every bucket B_j. */
    uint64_t start = 0;
    for (uint64_t j = 0; j < s; ++j) {
        qsort(out + start, bsz[j], sizeof(item_t), cmp_item);
        start += bsz[j];
    }

    /* R4: the pads are the order's maxima, so they occupy positions n .. np-1. */
    int status = ORACLE_OK;
    for (uint64_t t = n; t < np; ++t)
        if (out[t].idx < n) status = ORACLE_E_INVALID;
    for (uint64_t t = 0; t < n; ++t) {
        store_key(kind, keys_out, t, out[t].key);
        if (vals_out) vals_out[t] = out[t].val;
    }
    free(A); free(out); free(S); free(g); free(r); free(a); free(l); free(bsz);
    return status;
}
