"""GPU parity: the HIP pipeline (called through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact everywhere: final outputs, and the level-1 intermediates
of Algorithm 1 (sorted samples, global samples, a_ij, l_ij, bucket table) at the same (L, s),
on every configuration up to the full benchmark sizes (2^28 uint32 keys with the benchmark's own
plan, the six 2^26 distributions, 2^27 uint64 key/value pairs).  The oracle runs for the large
inputs are started on host threads when the module's first test runs, so they overlap the GPU
tests before them."""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_level1, from_dev, gpu_sort, oracle_pool, say, to_dev, ws_view

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def ds(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1002_4464_amd as d
    d.load_library()
    _start_heavy(d, {it.name for it in request.session.items})
    return d


C2_SEEDS = {"uniform": 2, "gaussian": 3, "bucket": 4, "staggered": 5, "sorted": 6, "equal": 7}
_HEAVY = {}


def _auto_plan(d, kt, values, n):
    g = d.Plan(kt, values, n).geometry(n)
    return g.sublist_len, g.samples


def _start_heavy(d, selected):
    """Submits the oracle runs of the large configurations whose tests are selected (each run
    generates its own copy of the seeded input, so the tests generate theirs for the GPU
    meanwhile)."""
    if _HEAVY:
        return
    pool = oracle_pool()

    def job(key, test, make, L, s, values=False):
        if test not in selected:
            return

        def run():
            keys = make()
            vals = synth.index_values(keys.size) if values else None
            return oracle.dss(keys, L, s, values=vals, trace=True, reloc=False)
        _HEAVY[key] = pool.submit(run)

    n28, n27, n26 = 1 << 28, 1 << 27, 1 << 26
    # the benchmark's plan: L = 16384, s = 256, 2^22 samples sorted in 8 merge rounds
    job("2p28", "test_headline_2p28_uniform", lambda: synth.uniform_u32(n28, 8), 16384, 256)
    L26, s26 = _auto_plan(d, 1, False, n26)
    for dist, seed in C2_SEEDS.items():
        job("2p26_" + dist, f"test_2p26_distributions[{dist}]",
            lambda dist=dist, seed=seed: synth.make_u32(dist, n26, seed), L26, s26)
    L27, s27 = _auto_plan(d, 2, True, n27)
    job("c3b_uniform", "test_2p27_u64_pairs[uniform]", lambda: synth.uniform_u64(n27, 9),
        L27, s27, values=True)
    job("c3b_zipf", "test_2p27_u64_pairs[zipf]", lambda: synth.zipf_u64(n27, 10), L27, s27,
        values=True)
    Lu, su = _auto_plan(d, 2, False, n26)
    job("u64_2p26", "test_two_level_u64_keys_2p26", lambda: synth.zipf_u64(n26, 17), Lu, su)


def _heavy(key):
    """The oracle result of one large configuration (released once taken)."""
    return _HEAVY.pop(key).result()


# ------------------------------------------------------------------ small, one tile

@pytest.mark.parametrize("n", [2, 3, 17, 64, 1000, 4097, 32767, 32768])
def test_single_tile_u32(ds, n):
    say(f"single tile u32 n={n}")
    keys = synth.uniform_u32(n, 100 + n) % np.uint32(max(2, n // 3))
    out, _, geo, _ = gpu_sort(ds, keys)
    assert geo.levels == 0
    assert (out == oracle.stable_sort(keys)[0]).all()


@pytest.mark.parametrize("kind", ["u32_pairs", "u64", "u64_pairs", "f32"])
def test_single_tile_types(ds, kind):
    say(f"single tile {kind}")
    n = 5000
    vals = synth.draws32(7, n)
    if kind.startswith("u64"):
        keys = synth.zipf_u64(n, 3, distinct=300)
    elif kind == "f32":
        keys = synth.normal_f32_segments([n], 4)
    else:
        keys = synth.uniform_u32(n, 5) % np.uint32(50)
    pv = vals if kind.endswith("pairs") else None
    out_k, out_v, geo, _ = gpu_sort(ds, keys, pv)
    ek, ev = oracle.stable_sort(keys, pv)
    assert geo.levels == 0
    assert (out_k.view(np.uint8) == ek.view(np.uint8)).all()
    if pv is not None:
        assert (out_v == ev).all()


# ------------------------------------------------------------------ one level, intermediates

def test_c1_uniform_2p20(ds):
    """2^20 uniform uint32 keys (seed 1), automatic plan: output and intermediates."""
    say("C1 2^20 uniform u32")
    keys = synth.uniform_u32(1 << 20, 1)
    out, _, geo, ws = gpu_sort(ds, keys)
    assert geo.levels == 1
    ok, _, tr = oracle.dss(keys, geo.sublist_len, geo.samples, trace=True)
    assert (out == ok).all()
    check_level1(geo, ws, tr, keys.size)


CASES = [
    # (n, L, s)
    (50_037, 1024, 32),
    (65_536, 2048, 64),
    (9_999, 256, 8),
    (100_003, 1024, 256),  # m*s > one workgroup: Step 4 by chunk sorts + merge rounds
    (16_385, 16384, 64),   # last sublist holds a single real item, the rest pads
    (200_003, 4096, 16),   # chunks of 256 items: ranks through the 16-item rank index
    (120_001, 16384, 16),  # chunks of 1024 items: 64 index entries per chunk, the most it takes
]


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_L{c[1]}_s{c[2]}")
def test_one_level_intermediates(ds, dist, case):
    n, L, s = case
    say(f"one level {dist} n={n} L={L} s={s}")
    keys = synth.make_u32(dist, n, 21)
    tu = ds.Tuning(L, s, 0, 0, 1)
    out, _, geo, ws = gpu_sort(ds, keys, tuning=tu)
    assert geo.levels == 1
    ok, _, tr = oracle.dss(keys, L, s, trace=True)
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


@pytest.mark.parametrize("kind", ["few_values", "descending"])
@pytest.mark.parametrize("L", [128, 256, 512, 1024, 4096])
def test_register_merge_levels(ds, L, kind):
    """Sublist lengths at which the 32-bit tile sort's in-register merges stop at runs of 128,
    256, 512 and 1024 items (one wave with 8, 16 or 32 active lanes for L = 128, 256, 512;
    whole waves from 1024), on inputs made of ties and key-max items or sorted the wrong way.
    The buckets (padded to multiples of 256) take every level count too.  Output and level-1
    intermediates against the oracle."""
    n = min(70_001, 70 * L + 17)  # about 70 sublists where smaller ones would not plan
    if kind == "few_values":
        table = np.array([0, 1, 0x7FFFFFFF, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32)
        keys = table[synth.draws32(77, n) % np.uint32(table.size)]
    else:
        keys = np.sort(synth.uniform_u32(n, 78))[::-1].copy()
    s = min(64, L // 8)
    say(f"register merge levels L={L} s={s} {kind}")
    out, _, geo, ws = gpu_sort(ds, keys, tuning=ds.Tuning(L, s, 0, 0, 1))
    assert geo.levels == 1 and geo.sublist_len == L
    ok, _, tr = oracle.dss(keys, L, s, trace=True)
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


def test_pairs_u32_stable_intermediates(ds):
    n = 300_001
    say(f"pairs u32 n={n}")
    keys = synth.uniform_u32(n, 31) % np.uint32(1000)
    vals = synth.index_values(n)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals)
    ok, ov, tr = oracle.dss(keys, geo.sublist_len, geo.samples, values=vals, trace=True)
    assert (out_k == ok).all() and (out_v == ov).all()
    check_level1(geo, ws, tr, n)


def test_f32_keys_intermediates(ds):
    sizes = [70_000]
    say("f32 keys n=70000 + specials")
    x = synth.normal_f32_segments(sizes, 41)
    x[::997] = np.float32(np.inf)
    x[5::1013] = np.float32(-np.inf)
    x[7::1021] = np.float32(np.nan)
    x[9::1031] = -np.float32(np.nan)
    out, _, geo, ws = gpu_sort(ds, x, tuning=ds.Tuning(2048, 32, 0, 0, 1))
    ok, _, tr = oracle.dss(x, 2048, 32, trace=True)
    assert (out.view(np.uint32) == ok.view(np.uint32)).all()
    check_level1(geo, ws, tr, x.size)


def test_f32_pairs(ds):
    n = 123_457
    say(f"f32 pairs n={n}")
    x = synth.normal_f32_segments([n], 43)
    vals = synth.index_values(n)
    out_k, out_v, geo, ws = gpu_sort(ds, x, vals)
    ok, ov, tr = oracle.dss(x, geo.sublist_len, geo.samples, values=vals, trace=True)
    assert (out_k.view(np.uint32) == ok.view(np.uint32)).all() and (out_v == ov).all()
    check_level1(geo, ws, tr, n)


@pytest.mark.parametrize("pairs", [False, True])
def test_u64_intermediates(ds, pairs):
    n = 200_003
    say(f"u64 pairs={pairs} n={n}")
    keys = synth.zipf_u64(n, 51, distinct=5000)
    vals = synth.index_values(n) if pairs else None
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals)
    ok, ov, tr = oracle.dss(keys, geo.sublist_len, geo.samples, values=vals, trace=True)
    assert (out_k == ok).all()
    if pairs:
        assert (out_v == ov).all()
    check_level1(geo, ws, tr, n)


def test_u64_pairs_global_sample_sort(ds):
    n = 400_000
    say(f"u64 pairs global sample sort n={n}")
    keys = synth.zipf_u64(n, 53, distinct=1000)
    vals = synth.index_values(n)
    tu = ds.Tuning(2048, 256, 0, 0, 1)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals, tuning=tu)
    assert geo.sample_sort_global
    ok, ov, tr = oracle.dss(keys, 2048, 256, values=vals, trace=True)
    assert (out_k == ok).all() and (out_v == ov).all()
    check_level1(geo, ws, tr, n)


# ------------------------------------------------------------------ two levels

@pytest.mark.parametrize("dist", ["uniform", "equal", "sorted", "staggered"])
def test_two_level_forced(ds, dist):
    n = 200_000 + 7
    say(f"two level forced {dist} n={n}")
    keys = synth.make_u32(dist, n, 61)
    tu = ds.Tuning(2048, 16, 1024, 0, 2)
    out, _, geo, ws = gpu_sort(ds, keys, tuning=tu)
    assert geo.levels == 2
    ok, _, tr = oracle.dss(keys, 2048, 16, trace=True)
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


def test_two_level_pairs_forced(ds):
    n = 150_001
    say(f"two level pairs n={n}")
    keys = synth.uniform_u32(n, 63) % np.uint32(77)
    vals = synth.index_values(n)
    tu = ds.Tuning(1024, 16, 512, 0, 2)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals, tuning=tu)
    assert geo.levels == 2
    ok, ov, tr = oracle.dss(keys, 1024, 16, values=vals, trace=True)
    assert (out_k == ok).all() and (out_v == ov).all()
    check_level1(geo, ws, tr, n)


def test_two_level_auto_2p24(ds):
    n = 1 << 24
    say(f"two level auto u32 n={n}")
    keys = synth.uniform_u32(n, 65)
    out, _, geo, ws = gpu_sort(ds, keys)
    assert geo.levels == 2
    ok, _, tr = oracle.dss(keys, geo.sublist_len, geo.samples, trace=True)
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


def test_module_sort_on_two_streams(ds):
    """The module-level ds.sort() keeps one plan per size class; two calls of one class enqueued
    on two streams at once each get their own stream's workspace, so both results match the
    oracle."""
    import torch
    n = 3_000_001
    inputs = [synth.uniform_u32(n, 91), synth.make_u32("bucket", n, 92)]
    wants = [oracle.stable_sort(k)[0] for k in inputs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        say(f"two streams, round {rep}")
        devs = [to_dev(k) for k in inputs]
        torch.cuda.synchronize()
        for t, st in zip(devs, streams):
            ds.sort(t, stream=st)
        torch.cuda.synchronize()
        for t, w in zip(devs, wants):
            assert (from_dev(t, np.uint32) == w).all()


@pytest.mark.parametrize("case", [
    # (key type, pairs, n, (L1, s1, L2, s2, levels)): sublist lengths that are not powers of two
    # (multiples of 64 items per thread) and sample counts that are not either (Step 4 then
    # starts from the largest power-of-two runs dividing s; chunks of the global sample sort
    # cut rows of s)
    (1, False, 300_007, (3072, 96, 0, 0, 1)),
    (1, False, 1_000_003, (15360, 320, 5120, 80, 2)),
    (2, True, 400_009, (7680, 640, 1536, 48, 2)),
], ids=["u32_one_L3072_s96", "u32_two_L15360_s320", "u64pairs_two_L7680_s640"])
def test_non_power_of_two_plans(ds, case):
    kt, pairs, n, t = case
    say(f"non-power-of-two plan kt={kt} pairs={pairs} n={n} tuning={t}")
    keys = synth.uniform_u32(n, 83) if kt == 1 else synth.zipf_u64(n, 84, distinct=1 << 14)
    vals = synth.index_values(n) if pairs else None
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals, tuning=ds.Tuning(*t))
    assert (geo.sublist_len, geo.samples, geo.levels) == (t[0], t[1], t[4])
    if t[4] == 2:
        assert (geo.sublist_len2, geo.samples2) == (t[2], t[3])
    ok, ov, tr = oracle.dss(keys, t[0], t[1], values=vals, trace=True)
    assert (out_k == ok).all()
    if pairs:
        assert (out_v == ov).all()
    check_level1(geo, ws, tr, n)


@pytest.mark.parametrize("kind", ["u32", "u64_pairs"])
def test_views_not_16_byte_aligned(ds, kind):
    """Keys (and values) starting one element past an aligned address: whole tiles then take
    the per-key loads and stores instead of the 128-bit ones, at both levels."""
    import torch
    n = 300_007
    say(f"unaligned views {kind} n={n}")
    if kind == "u32":
        keys, vals, kt, L = synth.uniform_u32(n, 85), None, 1, 4096
    else:
        keys, vals, kt, L = synth.zipf_u64(n, 86, distinct=1 << 12), synth.index_values(n), 2, 2048
    plan = ds.Plan(kt, vals is not None, n, ds.Tuning(L, 64, 0, 0, 2))
    tk = to_dev(np.concatenate([keys[:1], keys]))[1:]
    assert tk.data_ptr() % 16 != 0
    ws = plan.workspace(tk.device)
    if vals is None:
        plan.sort_keys(tk, ws)
        tv = None
    else:
        tv = to_dev(np.concatenate([vals[:1], vals]))[1:]
        assert tv.data_ptr() % 16 != 0
        plan.sort_pairs(tk, tv, ws)
    torch.cuda.synchronize()
    geo = plan.geometry(n)
    assert geo.levels == 2
    assert int(ws_view(ws, geo.off_status, 1, np.uint32)[0]) == 0
    ok, ov, tr = oracle.dss(keys, L, 64, values=vals, trace=True)
    assert (from_dev(tk, keys.dtype) == ok).all()
    if vals is not None:
        assert (from_dev(tv, np.uint32) == ov).all()
    check_level1(geo, ws, tr, n)


# ------------------------------------------------------------------ the headline plan's depth

@pytest.mark.parametrize("case", [
    # (key type, pairs, n, L, s): Step 4 runs the same number of global merge rounds as the
    # benchmark's 2^28 plan (8 rounds of 8-byte composites; 9 of 16-byte composites), at sizes
    # the oracle finishes in seconds
    (1, False, 1 << 25, 2048, 256),
    (2, True, 1 << 24, 1024, 256),
], ids=["u32_2p25_L2048_s256", "u64pairs_2p24_L1024_s256"])
def test_deep_sample_merge_intermediates(ds, case):
    kt, pairs, n, L, s = case
    say(f"deep sample merge kt={kt} pairs={pairs} n={n} L={L} s={s}")
    keys = synth.uniform_u32(n, 81) if kt == 1 else synth.zipf_u64(n, 82, distinct=1 << 16)
    vals = synth.index_values(n) if pairs else None
    fut = oracle_pool().submit(oracle.dss, keys, L, s, vals, True, False)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals, tuning=ds.Tuning(L, s, 0, 0, 2))
    assert geo.levels == 2 and geo.sample_sort_global
    ok, ov, tr = fut.result()
    assert (out_k == ok).all()
    if pairs:
        assert (out_v == ov).all()
    check_level1(geo, ws, tr, n)


# ------------------------------------------------------------------ benchmark sizes

def test_headline_2p28_uniform(ds):
    """The benchmark's configuration: 2^28 uniform uint32 keys (seed 8) with the automatic plan
    (L = 16384, s = 256, two levels, 2^22 samples sorted by chunk sorts and 8 merge rounds):
    every output key and every level-1 intermediate against the oracle at the same (L, s)."""
    n = 1 << 28
    say("2^28 uniform u32, benchmark plan")
    keys = synth.uniform_u32(n, 8)
    out, _, geo, ws = gpu_sort(ds, keys)
    assert (geo.levels, geo.sublist_len, geo.samples) == (2, 16384, 256)
    assert geo.sample_sort_global
    del keys
    ok, _, tr = _heavy("2p28")
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_2p26_distributions(ds, dist):
    """2^26 uint32 keys of each distribution (automatic plan): output and level-1
    intermediates against the oracle; a second run is bit-identical (determinism)."""
    n = 1 << 26
    say(f"2^26 {dist}")
    keys = synth.make_u32(dist, n, C2_SEEDS[dist])
    out, _, geo, ws = gpu_sort(ds, keys)
    out2, _, _, _ = gpu_sort(ds, keys)
    assert (out2 == out).all()
    ok, _, tr = _heavy("2p26_" + dist)
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_2p27_u64_pairs(ds, dist):
    """2^27 (uint64 key, uint32 value = input index), keys uniform (seed 9) or Zipf(1.1) over
    2^20 values (seed 10; its top key is about 12 % of the items): keys, values and level-1
    intermediates against the oracle's stable sort at the same (L, s)."""
    n = 1 << 27
    say(f"2^27 u64 pairs {dist}")
    keys = synth.uniform_u64(n, 9) if dist == "uniform" else synth.zipf_u64(n, 10)
    vals = synth.index_values(n)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals)
    assert geo.levels == 2
    del keys, vals
    ok, ov, tr = _heavy("c3b_" + dist)
    assert (out_k == ok).all() and (out_v == ov).all()
    check_level1(geo, ws, tr, n)


def test_two_level_f32_specials_2p25(ds):
    """Two levels on float32 keys with duplicates, signed zeros, infinities and NaNs of both
    signs: bit-exact against the oracle's stable sort (IEEE totalOrder)."""
    n = 1 << 25
    say("2^25 f32 two levels")
    x = synth.normal_f32_segments(np.array([n]), 14, dup_frac=0.01, zero_log2=8)
    bits = x.view(np.uint32).copy()
    pos = (synth.draws64(15, 4096) % np.uint64(n)).astype(np.int64)
    bits[pos] = np.resize(np.array([0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00001,
                                    0x80000000, 0x00000000], np.uint32), pos.size)
    keys = bits.view(np.float32)
    fut = oracle_pool().submit(oracle.stable_sort, keys)
    out, _, geo, _ = gpu_sort(ds, keys)
    assert geo.levels == 2
    want, _ = fut.result()
    assert (out.view(np.uint32) == want.view(np.uint32)).all()


def test_two_level_u32_pairs_duplicates_2p25(ds):
    """Two levels, 2^25 pairs over 256 distinct keys (every bucket boundary falls inside a run
    of equal keys): values bit-exact against the oracle's stable sort."""
    n = 1 << 25
    say("2^25 u32 pairs, 256 distinct keys")
    keys = (synth.draws32(16, n) & np.uint32(0xFF)).astype(np.uint32)
    vals = synth.index_values(n)
    fut = oracle_pool().submit(oracle.stable_sort, keys, vals)
    out_k, out_v, geo, _ = gpu_sort(ds, keys, vals)
    assert geo.levels == 2
    want_k, want_v = fut.result()
    assert (out_k == want_k).all() and (out_v == want_v).all()


def test_two_level_u64_keys_2p26(ds):
    """2^26 uint64 Zipf keys (seed 17), two levels: output and level-1 intermediates against
    the oracle."""
    n = 1 << 26
    say("2^26 u64 keys two levels")
    keys = synth.zipf_u64(n, 17)
    out, _, geo, ws = gpu_sort(ds, keys)
    assert geo.levels == 2
    ok, _, tr = _heavy("u64_2p26")
    assert (out == ok).all()
    check_level1(geo, ws, tr, n)


def _largest_plannable(ds, kt, values):
    lo, hi = 1 << 20, (1 << 32) - (1 << 16)
    while lo < hi:
        mid = (lo + hi + 1) // 2
        try:
            ds.Plan(kt, values, mid)
            lo = mid
        except ds.DsortError:
            hi = mid - 1
    return lo


@pytest.mark.timeout(900)
def test_largest_u32_sort(ds):
    """The largest uint32 sort a plan accepts (about 1.1e9 keys, 4.4 GB): output
    non-decreasing and the multiset unchanged (two 64-bit hashes summed over the array),
    checked on the device in chunks."""
    import torch
    n = _largest_plannable(ds, 1, False)
    say("largest u32 sort n =", n)
    assert n > 1 << 30
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    keys = torch.empty(n, dtype=torch.int32, device="cuda")
    chunk = 1 << 27

    def image(c):
        return c.to(torch.int64) & 0xFFFFFFFF

    def hashes():
        h1 = torch.zeros((), dtype=torch.int64, device="cuda")
        h2 = torch.zeros((), dtype=torch.int64, device="cuda")
        for a in range(0, n, chunk):
            x = image(keys[a:a + chunk])
            h1 += ((x * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) ^ (x >> 7)).sum()
            h2 += ((x ^ 0x5851F42D4C957F2D) * 0x2545F4914F6CDD1D).sum()
        return int(h1), int(h2)

    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        keys[a:a + m] = torch.randint(-(1 << 31), 1 << 31, (m,), dtype=torch.int64,
                                      device="cuda", generator=gen).to(torch.int32)
    before = hashes()
    plan = ds.Plan(1, False, n)
    ws = plan.workspace("cuda")
    plan.sort_keys(keys, ws)
    torch.cuda.synchronize()
    geo = plan.geometry(n)
    assert int(ws_view(ws, geo.off_status, 1, np.uint32)[0]) == 0
    for a in range(0, n, chunk):
        x = image(keys[a:min(n, a + chunk + 1)])
        assert bool((x[1:] >= x[:-1]).all()), f"order broken near {a}"
    assert hashes() == before
