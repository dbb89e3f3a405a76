"""GPU parity of the randomized-splitter variant (the comparison method that Sections 1 and 3
contrast with Algorithm 1): Step 3 of the first level takes s random sorted positions per sublist
and the last bucket is closed by +infinity.  The HIP path is compared element by element with
the oracle run with the same sampling and seed: the sorted output, and, where no bucket was
routed to the further run, the level-1 intermediates (sorted samples, a_ij, l_ij, bucket table).
Buckets that outgrow the normal path are forced by seeds found with the oracle, and the routed
count is checked against the oracle's bucket sizes."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from helpers import check_level1, from_dev, gpu_sort, oracle_pool, say, to_dev, ws_view

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ds():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1002_4464_amd as d
    d.load_library()
    return d


def rnd_tuning(ds, seed, L=0, s=0, L2=0, s2=0, levels=0):
    t = ds.Tuning(L, s, L2, s2, levels)
    t.sampling = 1
    t.seed = seed
    return t


def routed(geo, tr, n):
    """Level-1 buckets whose real size exceeds the normal path's limit (oracle sizes)."""
    begin = tr.offset[0].astype(np.int64)
    real = np.clip(n - begin, 0, tr.bucket_size.astype(np.int64))
    return int((real > geo.bucket_limit).sum())


def run_and_check(ds, keys, vals, tuning, seed, intermediates=True):
    plan = ds.Plan({np.dtype(np.uint32): 1, np.dtype(np.uint64): 2,
                    np.dtype(np.float32): 3}[keys.dtype], vals is not None, keys.size, tuning)
    geo0 = plan.geometry(keys.size)
    assert geo0.sampling == 1
    fut = oracle_pool().submit(oracle.dss, keys, geo0.sublist_len, geo0.samples, vals, True,
                               False, 1, seed)
    out_k, out_v, geo, ws = gpu_sort(ds, keys, vals, plan=plan)
    ok, ov, tr = fut.result()
    assert (out_k.view(np.uint8) == ok.view(np.uint8)).all(), "keys differ from the oracle"
    if vals is not None:
        assert (out_v == ov).all(), "values differ from the oracle"
    got = int(ws_view(ws, geo.off_overflow_count, 1, np.uint32)[0])
    want = routed(geo, tr, keys.size)
    assert got == want, f"routed buckets {got}, oracle sizes give {want}"
    if intermediates and want == 0:
        check_level1(geo, ws, tr, keys.size)
    return geo, want


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_random_one_level(ds, dist):
    n = 1_000_003
    say(f"random one level {dist} n={n}")
    seed = 1234
    geo, _ = run_and_check(ds, synth.make_u32(dist, n, 31), None, rnd_tuning(ds, seed), seed)
    assert geo.levels == 1


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_random_two_levels_2p24(ds, dist):
    n = 1 << 24
    say(f"random two levels {dist} n={n}")
    seed = 99
    geo, _ = run_and_check(ds, synth.make_u32(dist, n, 32), None, rnd_tuning(ds, seed), seed)
    assert geo.levels == 2


@pytest.mark.parametrize("dist", sorted(synth.DISTRIBUTIONS_U32))
def test_random_2p26_benchmark_plan(ds, dist):
    """The randomized runs the benchmark times: 2^26 uint32 keys of each distribution (seeds
    2-7), automatic plan, seed 2024; output and level-1 intermediates against the oracle."""
    n = 1 << 26
    seeds = {"uniform": 2, "gaussian": 3, "bucket": 4, "staggered": 5, "sorted": 6, "equal": 7}
    say(f"random 2^26 {dist}")
    geo, _ = run_and_check(ds, synth.make_u32(dist, n, seeds[dist]), None,
                           rnd_tuning(ds, 2024), 2024)
    assert geo.levels == 2


@pytest.mark.parametrize("kind", ["u32_pairs", "u64", "u64_pairs", "f32"])
def test_random_types(ds, kind):
    n = 300_001
    say(f"random {kind} n={n}")
    if kind.startswith("u64"):
        keys = synth.zipf_u64(n, 33, distinct=5000)
    elif kind == "f32":
        keys = synth.normal_f32_segments([n], 34)
        keys[::1009] = np.float32(-np.inf)
        keys[3::1013] = -np.float32(np.nan)
    else:
        keys = synth.uniform_u32(n, 35) % np.uint32(3000)
    vals = synth.index_values(n) if kind.endswith("pairs") else None
    seed = 7
    run_and_check(ds, keys, vals, rnd_tuning(ds, seed), seed)


def _find_routing_seed(keys, vals, L, s, limit, lo=1, tries=400):
    """First seed whose randomized buckets (oracle) include one above `limit`."""
    n = keys.size
    for seed in range(lo, lo + tries):
        _, _, tr = oracle.dss(keys, L, s, vals, True, False, 1, seed)
        begin = tr.offset[0].astype(np.int64)
        real = np.clip(n - begin, 0, tr.bucket_size.astype(np.int64))
        if (real > limit).any():
            return seed
    raise AssertionError("no seed routes a bucket; widen the search")


@pytest.mark.parametrize("case", [
    # (kind, n, L, s, L2, s2, levels): two or three sublists per bucket's worth of samples, so
    # random buckets often pass twice their mean, which is the normal path's limit
    ("u32_pairs", 32_765, 16384, 4, 0, 0, 1),
    ("f32_pairs", 32_765, 16384, 4, 0, 0, 1),
    ("u64", 32_767, 16384, 4, 0, 0, 1),
    ("u64_pairs", 16_381, 8192, 4, 0, 0, 1),
    ("u32_pairs", 49_001, 16384, 8, 1024, 2, 2),
    ("u32", 49_001, 16384, 8, 512, 1, 2),
], ids=lambda c: f"{c[0]}_n{c[1]}_lv{c[6]}")
def test_random_routed_buckets(ds, case):
    """Buckets beyond the normal path's limit are relocated as ranges and sorted by a further
    run: output against the oracle, routed count against the oracle's bucket sizes."""
    kind, n, L, s, L2, s2, levels = case
    if kind.startswith("u64"):
        keys = synth.zipf_u64(n, 40, distinct=n // 3)
    elif kind.startswith("f32"):
        keys = synth.normal_f32_segments([n], 41)
    else:
        keys = synth.uniform_u32(n, 42) % np.uint32(n // 2)
    vals = synth.index_values(n) if kind.endswith("pairs") else None
    kt = {"u32": 1, "u64": 2, "f32": 3}[kind[:3]]
    plan = ds.Plan(kt, vals is not None, n, rnd_tuning(ds, 1, L, s, L2, s2, levels))
    geo = plan.geometry(n)
    assert geo.levels == levels and geo.bucket_limit > 0
    seed = _find_routing_seed(keys, vals, L, s, geo.bucket_limit)
    say(f"random routed {kind} n={n} levels={levels} limit={geo.bucket_limit} seed={seed}")
    _, want = run_and_check(ds, keys, vals, rnd_tuning(ds, seed, L, s, L2, s2, levels), seed)
    assert want > 0


def test_random_repeatable(ds):
    """The same seed gives the same intermediates; another seed other buckets but the same
    (unique) sorted output."""
    n = 2_000_000
    say(f"random repeatable n={n}")
    keys = synth.make_u32("bucket", n, 43)
    a = gpu_sort(ds, keys, tuning=rnd_tuning(ds, 5))
    b = gpu_sort(ds, keys, tuning=rnd_tuning(ds, 5))
    c = gpu_sort(ds, keys, tuning=rnd_tuning(ds, 6))
    assert (a[0] == b[0]).all() and (a[0] == c[0]).all()
    geo = a[2]
    ca = ws_view(a[3], geo.off_counts, geo.sublists * geo.samples, np.uint32)
    cb = ws_view(b[3], geo.off_counts, geo.sublists * geo.samples, np.uint32)
    cc = ws_view(c[3], geo.off_counts, geo.sublists * geo.samples, np.uint32)
    assert (ca == cb).all() and not (ca == cc).all()


def test_random_refuses_capture(ds):
    """A randomized call reads back its routed buckets, so it refuses a capturing stream and
    enqueues nothing; the keys stay as they were."""
    import torch
    n = 100_000
    keys = synth.uniform_u32(n, 44)
    tk = to_dev(keys)
    plan = ds.Plan(1, False, n, rnd_tuning(ds, 3))
    ws = plan.workspace(tk.device)
    other = torch.zeros(1, device=tk.device)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        other.add_(1.0)  # the graph holds one kernel of its own
        rc = plan._lib.dsort_keys(plan._h, ctypes.c_void_p(tk.data_ptr()), n,
                                  ctypes.c_void_p(ws.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == ds.E_UNSUPPORTED
    torch.cuda.synchronize()
    assert (from_dev(tk, np.uint32) == keys).all()
