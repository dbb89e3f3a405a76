"""Pins for the CPU oracle (Algorithm 1, Section 4): it is checked against things other than
itself -- brute-force insertion sort, exhaustive tiny inputs, numpy's stable argsort, the bucket
bound the method guarantees, closed forms for sorted and all-equal inputs, the paper's own
parameter arithmetic and a hand-worked example.  CPU only."""
import itertools
import json
import os
import struct

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def insertion_sort(keys, vals=None):
    """Textbook stable insertion sort (strict comparison, so equal keys keep their order)."""
    k = list(keys)
    v = list(vals) if vals is not None else list(range(len(k)))
    for a in range(1, len(k)):
        x, y = k[a], v[a]
        b = a - 1
        while b >= 0 and k[b] > x:
            k[b + 1], v[b + 1] = k[b], v[b]
            b -= 1
        k[b + 1], v[b + 1] = x, y
    return k, v


def check_trace_invariants(tr, n):
    """Bucket-size guarantee of Section 4 (|B_j| <= 2n/s) in its exact form, plus the
    bookkeeping identities of Steps 6-7."""
    m, L, s = tr.m, tr.L, tr.s
    npad = m * L
    # Step 6: every sublist is cut into s pieces that cover it.
    assert (tr.count.sum(axis=1) == L).all()
    # Step 7: offsets are the bucket-major exclusive prefix sum, ending at n'.
    flat_c = tr.count.T.reshape(-1)
    flat_l = tr.offset.T.reshape(-1)
    assert flat_l[0] == 0
    assert (np.diff(flat_l.astype(np.int64)) == flat_c[:-1].astype(np.int64)).all()
    assert int(flat_l[-1] + flat_c[-1]) == npad
    # bucket sizes are column sums.
    assert (tr.bucket_size == tr.count.sum(axis=0)).all()
    # the guarantee: m <= |B_j| <= 2n'/s - m, and the last bucket holds at most n'/s.
    assert (tr.bucket_size >= m).all()
    assert (tr.bucket_size <= 2 * npad // s - m).all()
    assert tr.bucket_size[-1] <= npad // s
    # sorted samples are strictly increasing composites; global samples are S[j*m - 1].
    comp = list(zip(tr.sample_key.tolist(), tr.sample_pos.tolist()))
    assert all(a < b for a, b in zip(comp, comp[1:]))
    assert (tr.splitter_key == tr.sample_key[m - 1::m]).all()
    assert (tr.splitter_pos == tr.sample_pos[m - 1::m]).all()


# ------------------------------------------------------------------ hand-worked example

def test_worked_example(oracle_lib):
    """n=20, L=8, s=4 (w=2, m=3, n'=24).  Expected values were derived by hand from the
    definitions of Steps 1-9 under the readings listed in the oracle's header (chunk-end
    samples, splitters S[jm-1], (key, sublist, rank) tie-break, key-max pads)."""
    keys = np.array([5, 3, 9, 3, 3, 8, 1, 3, 3, 0, 9, 7, 3, 3, 2, 6, 4, 3, 9, 3], np.uint32)
    out, _, tr = oracle_lib.dss(keys, 8, 4, trace=True)
    P = 0xFFFFFFFF
    assert out.tolist() == [0, 1, 2, 3, 3, 3, 3, 3, 3, 3, 3, 3, 4, 5, 6, 7, 8, 9, 9, 9]
    # samples as (key, sublist, rank)
    samples = [(k, p // 8, p % 8) for k, p in zip(tr.sample_key.tolist(), tr.sample_pos.tolist())]
    assert samples == [(2, 1, 1), (3, 0, 1), (3, 0, 3), (3, 1, 3), (3, 2, 1), (5, 0, 5),
                       (6, 1, 5), (9, 0, 7), (9, 1, 7), (9, 2, 3), (P, 2, 5), (P, 2, 7)]
    splitters = [(k, p // 8, p % 8) for k, p in zip(tr.splitter_key.tolist(),
                                                    tr.splitter_pos.tolist())]
    assert splitters == [(3, 0, 3), (5, 0, 5), (9, 1, 7), (P, 2, 7)]
    assert tr.count.tolist() == [[4, 2, 2, 0], [2, 3, 3, 0], [0, 3, 0, 5]]
    assert tr.offset.tolist() == [[0, 6, 14, 19], [4, 8, 16, 19], [6, 11, 19, 19]]
    assert tr.bucket_size.tolist() == [6, 8, 5, 5]
    check_trace_invariants(tr, 20)


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("seed", range(40))
def test_against_insertion_sort_small(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    L = int(2 ** rng.integers(0, 8))
    s = int(2 ** rng.integers(0, int(np.log2(L)) + 1))
    hi = int(rng.choice([3, 50, 1 << 32]))
    keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    out_k, out_v, tr = oracle_lib.dss(keys, L, s, values=vals, trace=True)
    ek, ev = insertion_sort(keys.tolist(), vals.tolist())
    assert out_k.tolist() == ek
    assert out_v.tolist() == ev
    check_trace_invariants(tr, n)


def test_counts_equal_brute_force_definition(oracle_lib):
    """a_ij counted item by item against the splitters (no bisection, no rank rule)."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        n = int(rng.integers(1, 200))
        L = int(2 ** rng.integers(1, 6))
        s = int(2 ** rng.integers(0, int(np.log2(L)) + 1))
        keys = rng.integers(0, 6, size=n).astype(np.uint32)
        _, _, tr = oracle_lib.dss(keys, L, s, trace=True)
        m = tr.m
        padded = keys.tolist() + [0xFFFFFFFF] * (m * L - n)
        g = list(zip(tr.splitter_key.tolist(), tr.splitter_pos.tolist()))
        for i in range(m):
            sub = sorted(padded[i * L:(i + 1) * L])  # keys only: equal keys are interchangeable
            items = [(sub[r], i * L + r) for r in range(L)]
            for j in range(s):
                lo = g[j - 1] if j else None
                cnt = sum(1 for it in items if it <= g[j] and (lo is None or it > lo))
                assert cnt == tr.count[i, j]


@pytest.mark.parametrize("n", range(0, 8))
def test_exhaustive_ternary(oracle_lib, n):
    """Every array over {0, 1, 2} of length n, at several (L, s)."""
    shapes = [(1, 1), (2, 1), (2, 2), (4, 2), (4, 4), (8, 2)]
    for keys in itertools.product(range(3), repeat=n):
        arr = np.array(keys, np.uint32)
        expect, _ = insertion_sort(keys)
        for L, s in shapes:
            out, vals, tr = oracle_lib.dss(arr, L, s, values=np.arange(n, dtype=np.uint32),
                                           trace=True)
            assert out.tolist() == expect
            assert vals.tolist() == insertion_sort(keys)[1]
            if n:
                check_trace_invariants(tr, n)


# ------------------------------------------------------------------ library routine

@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_against_numpy_stable_argsort(oracle_lib, dist):
    n = (1 << 16) + 123
    keys = synth.make_u32(dist, n, 3)
    vals = synth.index_values(n)
    out_k, out_v, tr = oracle_lib.dss(keys, 1 << 10, 32, values=vals, trace=True)
    order = np.argsort(keys, kind="stable")
    assert (out_k == keys[order]).all()
    assert (out_v == vals[order]).all()
    check_trace_invariants(tr, n)


def test_uniform_2p20_against_numpy(oracle_lib):
    keys = synth.uniform_u32(1 << 20, 1)
    out, _, tr = oracle_lib.dss(keys, 1 << 14, 128, trace=True)
    assert (out == np.sort(keys)).all()
    check_trace_invariants(tr, 1 << 20)


def test_u64_zipf_pairs_stable(oracle_lib):
    n = 50_000
    keys = synth.zipf_u64(n, 10)
    vals = synth.index_values(n)
    out_k, out_v, tr = oracle_lib.dss(keys, 1 << 9, 16, values=vals, trace=True)
    order = np.argsort(keys, kind="stable")
    assert (out_k == keys[order]).all()
    assert (out_v == vals[order]).all()
    # stability stated directly: values increase inside every run of equal keys
    same = out_k[1:] == out_k[:-1]
    assert (out_v[1:][same] > out_v[:-1][same]).all()
    check_trace_invariants(tr, n)


def test_stable_sort_definition_against_numpy(oracle_lib):
    keys = synth.zipf_u64(10_000, 4)
    vals = synth.draws32(5, 10_000)
    k, v = oracle_lib.stable_sort(keys, vals)
    order = np.argsort(keys, kind="stable")
    assert (k == keys[order]).all() and (v == vals[order]).all()


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("dist", ["sorted", "equal"])
def test_closed_form_bucket_sizes(oracle_lib, dist):
    """Sorted and all-equal inputs give every bucket exactly n'/s items."""
    for n, L, s in [(1 << 14, 1 << 8, 16), ((1 << 14) - 37, 1 << 8, 32), (5000, 64, 8)]:
        keys = synth.make_u32(dist, n, 11)
        out, _, tr = oracle_lib.dss(keys, L, s, trace=True)
        assert (out == np.sort(keys)).all()
        npad = tr.m * L
        assert (tr.bucket_size == npad // s).all()
        check_trace_invariants(tr, n)


def test_degenerate_shapes(oracle_lib):
    keys = synth.uniform_u32(1000, 2)
    ref = np.sort(keys)
    # m = 1: one sublist, Step 2 alone sorts everything
    out, _, tr = oracle_lib.dss(keys, 1024, 8, trace=True)
    assert tr.m == 1 and (out == ref).all()
    assert (tr.offset[0] == np.concatenate([[0], np.cumsum(tr.count[0])[:-1]])).all()
    # s = 1: one bucket holding everything
    out, _, tr = oracle_lib.dss(keys, 64, 1, trace=True)
    assert tr.bucket_size.tolist() == [tr.m * 64] and (out == ref).all()
    # s = L: every item is a sample
    out, _, tr = oracle_lib.dss(keys, 16, 16, trace=True)
    assert (out == ref).all()
    check_trace_invariants(tr, 1000)
    # n = 0 and n = 1
    assert oracle_lib.dss(np.zeros(0, np.uint32), 8, 2)[0].size == 0
    assert oracle_lib.dss(np.array([7], np.uint32), 8, 2)[0].tolist() == [7]
    # key-max collisions with the pads
    keys = np.full(77, 0xFFFFFFFF, np.uint32)
    keys[::3] = 5
    out, vals, tr = oracle_lib.dss(keys, 16, 4, values=np.arange(77, dtype=np.uint32),
                                   trace=True)
    order = np.argsort(keys, kind="stable")
    assert (out == keys[order]).all() and (vals == order).all()
    check_trace_invariants(tr, 77)


def test_invalid_shapes_rejected(oracle_lib):
    keys = np.arange(10, dtype=np.uint32)
    for L, s in [(0, 1), (8, 0), (8, 3), (4, 8)]:
        with pytest.raises(ValueError):
            oracle_lib.dss(keys, L, s)


# ------------------------------------------------------------------ float32 order

def _total_order_key(bits):
    """IEEE 754-2008 totalOrder for binary32, written from its definition: sign first
    (negatives below positives), then magnitude (larger magnitude is lower when negative);
    NaN payloads order like magnitudes."""
    sign = bits >> 31
    mag = bits & 0x7FFFFFFF
    return (1, mag) if sign == 0 else (0, -mag)


def test_f32_total_order_image(oracle_lib):
    specials = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000,
                0x7F800001, 0xFF800001, 0x00000001, 0x80000001, 0x3F800000, 0xBF800000,
                0x7F7FFFFF, 0xFF7FFFFF, 0x7FFFFFFF, 0xFFFFFFFF]
    rng = np.random.default_rng(3)
    pats = specials + rng.integers(0, 1 << 32, size=2000, dtype=np.uint64).tolist()
    by_def = sorted(pats, key=_total_order_key)
    by_img = sorted(pats, key=oracle_lib.f32_order)
    assert by_def == by_img
    for p in pats:
        assert oracle_lib.f32_unorder(oracle_lib.f32_order(p)) == p
    # -0 < +0, -inf < finite < +inf, negative NaN lowest, positive NaN highest
    img = oracle_lib.f32_order
    assert img(0x80000000) < img(0x00000000)
    assert img(0xFFC00000) < img(0xFF800000) < img(0xBF800000) < img(0x3F800000) \
        < img(0x7F800000) < img(0x7FC00000)


def test_f32_dss_matches_total_order(oracle_lib):
    sizes = synth.segment_sizes(3, 11, 8, 12)
    x = synth.normal_f32_segments(sizes, 11)
    x = np.concatenate([x, np.array([np.inf, -np.inf, np.nan, -np.nan, 0.0, -0.0] * 5,
                                    np.float32)])
    bits = x.view(np.uint32)
    out, vals, _ = oracle_lib.dss(x, 256, 16, values=np.arange(x.size, dtype=np.uint32))
    order = sorted(range(x.size), key=lambda t: (_total_order_key(int(bits[t])), t))
    assert out.view(np.uint32).tolist() == bits[order].tolist()
    assert vals.tolist() == order


# ------------------------------------------------------------------ the paper's parameters

@pytest.mark.slow
def test_paper_parameters(oracle_lib):
    """The paper's configuration: n = 32M, n/m = 2K, s = 64 (Section 4)."""
    with open(os.path.join(GOLDEN, "paper_section4_parameters.json")) as f:
        p = json.load(f)
    n, L, s = p["n"], p["sublist_len"], p["s"]
    assert n // L == p["m"]
    assert L // p["threads_per_block"] == p["items_per_thread"]
    assert s * p["m"] == p["sm"]
    assert 2 ** p["search_rounds"] == s
    keys = synth.uniform_u32(n, 8)
    out, _, tr = oracle_lib.dss(keys, L, s, trace=True)
    assert tr.m == p["m"] and tr.sample_key.size == p["sm"]
    assert tr.bucket_size.max() <= p["bucket_bound_2n_over_s"]
    assert (out == np.sort(keys)).all()
    check_trace_invariants(tr, n)


# ------------------------------------------------------------------ batches of sorts

def test_segmented_sort_definition(oracle_lib):
    """A batch of sorts: each segment independently equals numpy's stable sort of that range;
    gaps between segments, empty and one-item segments are left as they are."""
    n = 20_000
    keys = synth.make_u32("bucket", n, 21)
    vals = synth.index_values(n)
    offsets = [0, 0, 1, 700, 700, 5000, 5003, 9000, 19_999]  # [9000, 19_999) sorted, tail not
    k, v = oracle_lib.segmented_sort(keys, offsets, vals)
    for lo, hi in zip(offsets[:-1], offsets[1:]):
        order = np.argsort(keys[lo:hi], kind="stable")
        assert (k[lo:hi] == keys[lo:hi][order]).all()
        assert (v[lo:hi] == vals[lo:hi][order]).all()
    assert k[-1] == keys[-1] and v[-1] == vals[-1]
    # float32 segments under the total order, duplicates and signed zeros included
    sizes = synth.segment_sizes(6, 4, 2, 11)
    x = synth.normal_f32_segments(sizes, 4, dup_frac=0.05, zero_log2=4)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    k, _ = oracle_lib.segmented_sort(x, offs)
    for lo, hi in zip(offs[:-1], offs[1:]):
        want = sorted(x[lo:hi].view(np.uint32).tolist(), key=_total_order_key)
        assert k[lo:hi].view(np.uint32).tolist() == want
    with pytest.raises(ValueError):
        oracle_lib.segmented_sort(keys, [0, 10, 5])
    with pytest.raises(ValueError):
        oracle_lib.segmented_sort(keys, [0, n + 1])


# ------------------------------------------------------------------ randomized splitters (R8)
#
# The comparison method of Sections 1 and 3 builds its buckets from randomly selected items.
# The oracle's randomized variant takes Step 3's samples at random sorted positions drawn from
# its own SplitMix64 stream and closes the last bucket by +infinity; everything else is
# Algorithm 1 unchanged.  Its result is still the unique sorted order; its buckets have no
# bound.


def test_splitmix64_published_outputs(oracle_lib):
    """The oracle's generator and the input generator (two independent implementations of the
    published definition) both reproduce the reference implementation's first outputs."""
    with open(os.path.join(GOLDEN, "splitmix64_vectors.json")) as f:
        gold = json.load(f)
    for stream in gold["streams"]:
        want = [int(x) for x in stream["outputs"]]
        got = [oracle_lib.splitmix64(stream["seed"], c) for c in range(len(want))]
        assert got == want
        assert synth.draws64(stream["seed"], len(want)).tolist() == want


def _random_positions(seed, m, s, L):
    """Sample positions i*L + r of the randomized variant, computed with numpy from the input
    generator's draws (not the oracle's): draw i*s + k, top 32 bits times L, shifted down."""
    d = synth.draws64(seed, m * s) >> np.uint64(32)
    r = (d * np.uint64(L)) >> np.uint64(32)
    return r.reshape(m, s) + (np.arange(m, dtype=np.uint64) * np.uint64(L))[:, None]


def check_random_trace(tr, keys, seed):
    """Bookkeeping of the randomized variant: the samples are the items at the drawn positions,
    sorted; each bucket holds exactly m samples; the last bucket is closed by +infinity; Steps
    6-7 identities as for Algorithm 1."""
    m, L, s = tr.m, tr.L, tr.s
    pos = _random_positions(seed, m, s, L)
    assert sorted(tr.sample_pos.tolist()) == sorted(pos.reshape(-1).tolist())
    padded = np.concatenate([keys.astype(np.uint64),
                             np.full(m * L - keys.size, np.iinfo(keys.dtype).max, np.uint64)])
    comp = list(zip(tr.sample_key.tolist(), tr.sample_pos.tolist()))
    assert all(a <= b for a, b in zip(comp, comp[1:]))
    # the sample at position p holds the p-th smallest item of its sublist (stable order)
    for i in range(m):
        sub = np.sort(padded[i * L:(i + 1) * L], kind="stable")
        mine = tr.sample_pos >= np.uint64(i * L)
        mine &= tr.sample_pos < np.uint64((i + 1) * L)
        r = (tr.sample_pos[mine] - np.uint64(i * L)).astype(np.int64)
        assert (tr.sample_key[mine] == sub[r]).all()
    assert (tr.count.sum(axis=1) == L).all()
    flat_c = tr.count.T.reshape(-1)
    flat_l = tr.offset.T.reshape(-1)
    assert flat_l[0] == 0
    assert (np.diff(flat_l.astype(np.int64)) == flat_c[:-1].astype(np.int64)).all()
    assert int(flat_l[-1] + flat_c[-1]) == m * L
    assert (tr.bucket_size == tr.count.sum(axis=0)).all()
    # samples per bucket: bucket j < s is (g_{j-1}, g_j] with g_j = S[jm - 1]; bucket s is
    # everything above g_{s-1}.  Each holds exactly m samples when no position was drawn twice
    # (a repeated position repeats its sample, and equal samples share a bucket).
    if len(set(comp)) < len(comp):
        return
    for j in range(s):
        lo = comp[j * m - 1] if j else None
        hi = comp[(j + 1) * m - 1] if j + 1 < s else None
        inside = [c for c in comp if (lo is None or c > lo) and (hi is None or c <= hi)]
        assert len(inside) == m


@pytest.mark.parametrize("seed", range(40))
def test_random_against_insertion_sort_small(oracle_lib, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 400))
    L = int(2 ** rng.integers(0, 8))
    s = int(2 ** rng.integers(0, int(np.log2(L)) + 1))
    hi = int(rng.choice([3, 50, 1 << 32]))
    keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    vals = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    out_k, out_v, tr = oracle_lib.dss(keys, L, s, values=vals, trace=True, sampling=1,
                                      seed=seed)
    ek, ev = insertion_sort(keys.tolist(), vals.tolist())
    assert out_k.tolist() == ek
    assert out_v.tolist() == ev
    check_random_trace(tr, keys, seed)


def test_random_counts_equal_brute_force_definition(oracle_lib):
    """a_ij of the randomized variant counted item by item: bucket j < s holds the items in
    (g_{j-1}, g_j], bucket s every item above g_{s-1}."""
    rng = np.random.default_rng(8)
    for t in range(30):
        n = int(rng.integers(1, 200))
        L = int(2 ** rng.integers(1, 6))
        s = int(2 ** rng.integers(0, int(np.log2(L)) + 1))
        keys = rng.integers(0, 6, size=n).astype(np.uint32)
        _, _, tr = oracle_lib.dss(keys, L, s, trace=True, sampling=1, seed=t)
        m = tr.m
        padded = keys.tolist() + [0xFFFFFFFF] * (m * L - n)
        comp = list(zip(tr.sample_key.tolist(), tr.sample_pos.tolist()))
        g = [comp[(j + 1) * m - 1] for j in range(s - 1)]
        for i in range(m):
            sub = sorted(padded[i * L:(i + 1) * L])
            items = [(sub[r], i * L + r) for r in range(L)]
            for j in range(s):
                lo = g[j - 1] if j else None
                hi = g[j] if j + 1 < s else None
                cnt = sum(1 for it in items
                          if (lo is None or it > lo) and (hi is None or it <= hi))
                assert cnt == tr.count[i, j]


@pytest.mark.parametrize("n", range(1, 7))
def test_random_exhaustive_ternary(oracle_lib, n):
    shapes = [(1, 1), (2, 2), (4, 2), (4, 4), (8, 2)]
    for keys in itertools.product(range(3), repeat=n):
        arr = np.array(keys, np.uint32)
        expect, order = insertion_sort(keys)
        for L, s in shapes:
            for seed in (0, 5):
                out, vals, tr = oracle_lib.dss(arr, L, s, values=np.arange(n, dtype=np.uint32),
                                               trace=True, sampling=1, seed=seed)
                assert out.tolist() == expect
                assert vals.tolist() == order
                check_random_trace(tr, arr, seed)


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_random_against_numpy_stable_argsort(oracle_lib, dist):
    n = (1 << 16) + 123
    keys = synth.make_u32(dist, n, 40)
    vals = synth.index_values(n)
    out_k, out_v, tr = oracle_lib.dss(keys, 1024, 32, values=vals, trace=True, sampling=1,
                                      seed=77)
    order = np.argsort(keys, kind="stable")
    assert (out_k == keys[order]).all() and (out_v == order).all()
    check_random_trace(tr, keys, 77)


def test_random_buckets_have_no_bound(oracle_lib):
    """Random samples give no bucket guarantee: with one sublist (m = 1) some seed puts more
    than 2n'/s - m items into one bucket, which the equidistant samples never do."""
    keys = synth.uniform_u32(64, 9)
    L, s = 64, 8
    worst = 0
    for seed in range(64):
        _, _, tr = oracle_lib.dss(keys, L, s, trace=True, sampling=1, seed=seed)
        worst = max(worst, int(tr.bucket_size.max()))
    assert worst > 2 * 64 // s - 1
    _, _, tr = oracle_lib.dss(keys, L, s, trace=True)
    assert int(tr.bucket_size.max()) <= 2 * 64 // s - 1
