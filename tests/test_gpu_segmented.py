"""GPU parity of the segmented sort (many independent sorts in one call) against the oracle.

Every segment's result is unique (a sort, stable for key/value pairs), so the bar is bit-exact
against ``oracle.segmented_sort`` on the same seeded input: segment sizes on both sides of every
size-class capacity and of the one-workgroup limit, empty and one-item segments, gaps between
segments (left untouched), float32 duplicates, signed zeros and NaNs, up to the full batched
workload (4096 float32 segments, sizes log-uniform in [2^8, 2^20]), where every segment is
compared with the oracle."""
import numpy as np
import pytest

import oracle
import synth
from helpers import from_dev, oracle_pool, oracle_segmented, say, to_dev, ws_view

pytestmark = pytest.mark.gpu

KT = {np.dtype(np.uint32): 1, np.dtype(np.uint64): 2, np.dtype(np.float32): 3}


@pytest.fixture(scope="module")
def ds():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1002_4464_amd as d
    d.load_library()
    return d


def gpu_segmented(ds, keys, offsets, values=None, max_segment=0, plan=None, expect_status=0):
    import torch
    offsets = np.asarray(offsets, dtype=np.int64)
    S = offsets.size - 1
    if plan is None:
        plan = ds.Plan(KT[keys.dtype], values is not None, max(keys.size, 2), max_segments=S)
    tk = to_dev(keys)
    to = torch.from_numpy(offsets.copy()).cuda()
    tv = to_dev(values) if values is not None else None
    ws = plan.workspace(tk.device)
    plan.sort_segmented(tk, to, tv, max_segment=max_segment, workspace=ws)
    torch.cuda.synchronize()
    geo = plan.segmented_geometry(keys.size, S, max_segment)
    status = int(ws_view(ws, geo.off_status, 1, np.uint32)[0])
    assert status == expect_status, f"kernel status flags {status:#x}"
    out_v = from_dev(tv, np.uint32) if tv is not None else None
    return from_dev(tk, keys.dtype), out_v, geo


def offsets_of(sizes, gaps=None):
    """CSR offsets for consecutive segments; gaps[g] items left out before segment g."""
    offs = [0]
    pos = 0
    for g, z in enumerate(sizes):
        if gaps is not None:
            pos += int(gaps[g])
        if g == 0:
            offs[0] = pos
        else:
            offs.append(pos)
        pos += int(z)
    offs.append(pos)
    return np.array(offs, dtype=np.int64), pos


def mixed_u32(sizes, seed):
    dists = list(synth.DISTRIBUTIONS_U32)
    parts = [synth.make_u32(dists[g % len(dists)], int(z), seed + g) for g, z in enumerate(sizes)]
    return np.concatenate(parts) if parts else np.zeros(0, np.uint32)


# Sizes around the class capacities and the one-workgroup limit of each layout.
EDGE_U32 = [0, 1, 2, 3, 63, 64, 65, 2047, 2048, 2049, 4096, 6144, 8191, 8193, 12288, 16383,
            16384, 16385, 32767, 32768, 32769, 32769 + 16384, 49153, 65536, 100_003, 0, 1]


def test_u32_keys_edge_sizes(ds):
    sizes = EDGE_U32 + [(1 << 20) + 17]
    gaps = [(g * 37) % 5 for g in range(len(sizes))]
    offs, total = offsets_of(sizes, gaps)
    n = total + 11  # a tail outside every segment
    keys = mixed_u32([n], 3)
    keys[: total] = mixed_u32([total], 5)
    say("[seg] u32 keys", len(sizes), "segments, n =", n)
    out, _, geo = gpu_segmented(ds, keys, offs)
    want, _ = oracle.segmented_sort(keys, offs)
    assert geo.classes == 1 and geo.max_long_segments[0] > 0
    assert (out == want).all()


@pytest.mark.parametrize("dist", list(synth.DISTRIBUTIONS_U32))
def test_u32_keys_distributions(ds, dist):
    sizes = synth.segment_sizes(48, 100 + len(dist), 8, 19)
    offs, n = offsets_of(sizes)
    keys = synth.make_u32(dist, n, 17)
    say("[seg] u32", dist, "n =", n)
    out, _, _ = gpu_segmented(ds, keys, offs)
    want, _ = oracle.segmented_sort(keys, offs)
    assert (out == want).all()


def test_u32_pairs_stable(ds):
    sizes = [0, 1, 5, 1000, 4095, 4097, 8192, 16383, 16384, 16385, 40_000, 300_001, 2, 16384 * 3]
    offs, n = offsets_of(sizes, [3] * len(sizes))
    keys = (synth.draws32(7, n) & np.uint32(0xFF)).astype(np.uint32)  # many equal keys
    vals = synth.index_values(n)
    say("[seg] u32 pairs n =", n)
    out_k, out_v, _ = gpu_segmented(ds, keys, offs, vals)
    want_k, want_v = oracle.segmented_sort(keys, offs, vals)
    assert (out_k == want_k).all()
    assert (out_v == want_v).all()


def test_f32_keys_specials(ds):
    sizes = synth.segment_sizes(64, 9, 8, 18)
    sizes[3] = 0
    sizes[4] = 1
    offs, n = offsets_of(sizes)
    x = synth.normal_f32_segments(sizes, 9, dup_frac=0.01, zero_log2=10)
    bits = x.view(np.uint32).copy()
    rng_pos = synth.draws64(91, 64) % np.uint64(n)
    specials = np.array([0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000, 0x80000000, 0,
                         0x00000001, 0x80000001], np.uint32)
    bits[rng_pos.astype(np.int64)] = np.resize(specials, 64)
    keys = bits.view(np.float32)
    say("[seg] f32 n =", n)
    out, _, _ = gpu_segmented(ds, keys, offs)
    want, _ = oracle.segmented_sort(keys, offs)
    assert (out.view(np.uint32) == want.view(np.uint32)).all()


def test_f32_pairs(ds):
    sizes = synth.segment_sizes(40, 12, 6, 18)
    offs, n = offsets_of(sizes)
    keys = synth.normal_f32_segments(sizes, 12, dup_frac=0.2, zero_log2=3)
    vals = synth.index_values(n)
    out_k, out_v, _ = gpu_segmented(ds, keys, offs, vals)
    want_k, want_v = oracle.segmented_sort(keys, offs, vals)
    assert (out_k.view(np.uint32) == want_k.view(np.uint32)).all()
    assert (out_v == want_v).all()


@pytest.mark.parametrize("pairs", [False, True])
def test_u64_zipf(ds, pairs):
    sizes = [0, 1, 777, 8191, 8192, 8193, 16383, 16384, 16385, 70_000, 250_000, 3]
    offs, n = offsets_of(sizes, [1] * len(sizes))
    keys = synth.zipf_u64(n, 23)
    vals = synth.index_values(n) if pairs else None
    say("[seg] u64 pairs" if pairs else "[seg] u64 keys", "n =", n)
    out_k, out_v, _ = gpu_segmented(ds, keys, offs, vals)
    want_k, want_v = oracle.segmented_sort(keys, offs, vals)
    assert (out_k == want_k).all()
    if pairs:
        assert (out_v == want_v).all()


def test_tight_bound_same_result(ds):
    """A tight max_segment (fewer samples per sublist) gives the same, unique result."""
    sizes = synth.segment_sizes(30, 31, 10, 17)
    offs, n = offsets_of(sizes)
    keys = synth.uniform_u32(n, 31)
    plan = ds.Plan(1, False, n, max_segments=len(sizes))
    g_loose = plan.segmented_geometry(n, len(sizes), 0)
    g_tight = plan.segmented_geometry(n, len(sizes), int(sizes.max()))
    assert g_tight.samples[0] <= g_loose.samples[0]
    a, _, _ = gpu_segmented(ds, keys, offs, plan=plan)
    b, _, _ = gpu_segmented(ds, keys, offs, plan=plan, max_segment=int(sizes.max()))
    want, _ = oracle.segmented_sort(keys, offs)
    assert (a == want).all() and (b == want).all()


def test_plan_reuse_many_calls(ds):
    """One plan and workspace serve consecutive calls with different batches."""
    plan = ds.Plan(1, False, 1 << 21, max_segments=512)
    for seed in range(3):
        sizes = synth.segment_sizes(100 + 150 * seed, 40 + seed, 4, 15)
        offs, n = offsets_of(sizes)
        keys = synth.uniform_u32(n, seed)
        out, _, _ = gpu_segmented(ds, keys, offs, plan=plan)
        want, _ = oracle.segmented_sort(keys, offs)
        assert (out == want).all()


def test_invalid_offsets_flagged(ds):
    """Bad offsets are caught on the device.  Offsets that decrease or run past n (segments
    that would overlap or leave the array): nothing is sorted, status flag 0x10.  A segment
    longer than the stated max_segment: that segment stays as it is, the others are sorted, flag
    0x20."""
    n = 200_000
    keys = synth.uniform_u32(n, 77)
    plan = ds.Plan(1, False, n, max_segments=4)
    for offs in ([0, 1000, 500, 90_000], [0, 1000, 90_000, n + 5]):
        out, _, _ = gpu_segmented(ds, keys, np.array(offs), plan=plan, expect_status=16)
        assert (out == keys).all()
    offs = np.array([0, 100, 100_000, 150_000, 190_000], dtype=np.int64)
    out, _, _ = gpu_segmented(ds, keys, offs, max_segment=60_000, plan=plan, expect_status=32)
    for lo, hi in [(0, 100), (100_000, 150_000), (150_000, 190_000)]:
        assert (out[lo:hi] == oracle.stable_sort(keys[lo:hi])[0]).all()
    assert (out[100:100_000] == keys[100:100_000]).all()
    assert (out[190_000:] == keys[190_000:]).all()
    # the same plan and workspace then serve a clean call normally
    out, _, _ = gpu_segmented(ds, keys, offs, plan=plan)
    want, _ = oracle.segmented_sort(keys, offs)
    assert (out == want).all()


def test_abi_errors(ds):
    import torch
    plan = ds.Plan(1, False, 1 << 16, max_segments=4)
    k = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    o = torch.tensor([0, 10, 20, 30, 40, 50], dtype=torch.int64, device="cuda")
    with pytest.raises(ds.DsortError) as e:  # 5 segments > plan's 4
        plan.sort_segmented(k, o)
    assert e.value.status == ds.E_INVALID
    big = ds.Plan(1, False, 1 << 23, max_segments=4)
    k2 = torch.zeros(1 << 23, dtype=torch.int32, device="cuda")
    with pytest.raises(ds.DsortError) as e:  # a bound above the one-level limit
        big.sort_segmented(k2, o[:5], max_segment=(1 << 22))
    assert e.value.status == ds.E_UNSUPPORTED
    with pytest.raises(ValueError):
        plan.sort_segmented(k, o[:5], values=k)
    # empty batch and empty array are no-ops
    plan.sort_segmented(k, o[:1])
    torch.cuda.synchronize()


@pytest.mark.timeout(600)
def test_full_batched_workload(ds):
    """4096 float32 segments of sizes log-uniform in [2^8, 2^20] (about 5.1e8 keys), the batched
    benchmark workload: every segment bit-exact against the oracle (computed on host threads
    while the GPU sorts)."""
    import torch
    sizes = synth.segment_sizes(4096, 4, 8, 20)
    offs, n = offsets_of(sizes)
    say("[seg] full batched workload: generating", n, "keys")
    x = synth.normal_f32_segments(sizes, 4)
    S = sizes.size
    fut = oracle_pool().submit(oracle_segmented, x, offs)
    plan = ds.Plan(3, False, n, max_segments=S)
    tk = to_dev(x)
    to = torch.from_numpy(offs).cuda()
    ws = plan.workspace(tk.device)
    say("[seg] sorting")
    plan.sort_segmented(tk, to, max_segment=int(sizes.max()), workspace=ws)
    torch.cuda.synchronize()
    geo = plan.segmented_geometry(n, S, int(sizes.max()))
    assert int(ws_view(ws, geo.off_status, 1, np.uint32)[0]) == 0
    got = from_dev(tk, np.uint32)
    del tk, ws
    say("[seg] waiting for the oracle")
    want, _ = fut.result()
    bad = np.flatnonzero(got != want.view(np.uint32))
    assert bad.size == 0, f"{bad.size} keys differ, first at {bad[:4]}"


def _tuning(ds, upper, L, s):
    t = ds.SegTuning()
    t.classes = len(upper)
    for i in range(len(upper)):
        t.upper[i], t.sublist_len[i], t.samples[i] = upper[i], L[i], s[i]
    return t


@pytest.mark.parametrize("kt,pairs", [(1, False), (1, True), (2, True), (3, False)])
def test_tuned_classes_parity(ds, kt, pairs):
    """Long segments split into four length classes, each with its own sublist length and
    samples per sublist (including non-default ones), sort to the oracle's result; segment
    lengths sit on both sides of every class bound."""
    dt = {1: np.uint32, 2: np.uint64, 3: np.float32}[kt]
    probe = ds.Plan(kt, pairs, 1 << 16, max_segments=1)
    cap = probe.segmented_geometry(1 << 16, 1).small_capacity
    lim = probe.segmented_geometry(1 << 16, 1).segment_limit
    upper = [cap * 4, cap * 16, cap * 64, 1 << 62]
    sizes = [0, 5, cap, cap + 1, 3 * cap, cap * 4, cap * 4 + 1, cap * 10, cap * 16,
             cap * 16 + 7, min(lim, cap * 40), 77, min(lim, cap * 64 + 1)]
    offs, n = offsets_of(sizes, [2] * len(sizes))
    n += 3
    if kt == 3:
        keys = synth.normal_f32_segments(np.array([n]), 41, dup_frac=0.05, zero_log2=8)
    elif kt == 2:
        keys = synth.zipf_u64(n, 41)
    else:
        keys = synth.make_u32("bucket", n, 41)
    vals = synth.index_values(n) if pairs else None
    plan = ds.Plan(kt, pairs, n, max_segments=len(sizes))
    tl = plan.segmented_geometry(n, len(sizes)).sublist_len[0]
    Ls = [tl // 8, tl // 4, tl, tl]
    plan.set_seg_tuning(_tuning(ds, upper, Ls, [0, 0, 0, 0]))
    geo = plan.segmented_geometry(n, len(sizes))
    say("[seg] tuned classes", kt, pairs, "n =", n, "L =", geo.sublist_len, "s =", geo.samples)
    assert geo.classes >= 3
    out_k, out_v, _ = gpu_segmented(ds, keys, offs, vals, plan=plan)
    want_k, want_v = oracle.segmented_sort(keys, offs, vals)
    assert (out_k.view(np.uint8) == want_k.view(np.uint8)).all()
    if pairs:
        assert (out_v == want_v).all()
    # doubled samples per sublist in the two shorter classes: same result
    t = _tuning(ds, upper, Ls, [2 * geo.samples[0], 2 * geo.samples[1], 0, 0])
    plan.set_seg_tuning(t)
    out_k2, out_v2, _ = gpu_segmented(ds, keys, offs, vals, plan=plan)
    assert (out_k2.view(np.uint8) == want_k.view(np.uint8)).all()
    if pairs:
        assert (out_v2 == want_v).all()


def test_autotune_installs_and_keeps_input(ds):
    """The autotuner leaves the batch unchanged, installs a feasible tuning per length class,
    and sorts under it give the oracle's result."""
    import torch
    sizes = synth.segment_sizes(200, 61, 8, 20)
    offs, n = offsets_of(sizes)
    keys = synth.uniform_u32(n, 61)
    plan = ds.Plan(1, False, n, max_segments=sizes.size)
    tk = to_dev(keys)
    to = torch.from_numpy(offs).cuda()
    t = plan.autotune_segmented(tk, to, max_segment=int(sizes.max()), repeats=2)
    torch.cuda.synchronize()
    say("[seg] autotuned", t.as_dict())
    assert (from_dev(tk, np.uint32) == keys).all(), "autotuning must not touch the batch"
    assert t.classes >= 1 and plan.seg_tuning().as_dict() == t.as_dict()
    assert all(L > 0 and s > 0 for L, s in zip(t.as_dict()["sublist_len"],
                                                t.as_dict()["samples"]))
    out, _, _ = gpu_segmented(ds, keys, offs, plan=plan, max_segment=int(sizes.max()))
    want, _ = oracle.segmented_sort(keys, offs)
    assert (out == want).all()


def test_autotune_cache_file(ds, tmp_path, monkeypatch):
    """With DSORT_TUNE_CACHE set, a tuning is stored under (device, layout, segment class); a
    second autotune call for another batch of the same class installs it without timing and
    sorts under it still give the oracle's result."""
    import torch
    path = tmp_path / "dsort_tune.txt"
    monkeypatch.setenv("DSORT_TUNE_CACHE", str(path))
    sizes = synth.segment_sizes(150, 62, 8, 19)
    offs, n = offsets_of(sizes)
    keys = synth.uniform_u32(n, 62)
    plan = ds.Plan(1, False, n, max_segments=sizes.size)
    t1 = plan.autotune_segmented(to_dev(keys), torch.from_numpy(offs).cuda(),
                                 max_segment=int(sizes.max()), repeats=1)
    torch.cuda.synchronize()
    assert t1.from_cache == 0
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("v1 ")
    # another batch of the same longest-segment class, on a new plan
    sizes2 = synth.segment_sizes(150, 63, 8, 19)
    sizes2[0] = int(sizes.max())
    offs2, n2 = offsets_of(sizes2)
    keys2 = synth.normal_f32_segments(sizes2, 64).view(np.uint32)
    plan2 = ds.Plan(1, False, max(n, n2), max_segments=sizes2.size)
    t2 = plan2.autotune_segmented(to_dev(keys2), torch.from_numpy(offs2).cuda(),
                                  max_segment=int(sizes2.max()), repeats=1)
    torch.cuda.synchronize()
    say("[seg] cached tuning", t2.as_dict())
    assert t2.from_cache == 1 and t2.as_dict() == t1.as_dict()
    assert plan2.seg_tuning().as_dict() == t1.as_dict()
    assert len(path.read_text().splitlines()) == 1
    out, _, _ = gpu_segmented(ds, keys2, offs2, plan=plan2, max_segment=int(sizes2.max()))
    want, _ = oracle.segmented_sort(keys2, offs2)
    assert (out == want).all()


def test_concurrent_calls_from_two_threads(ds):
    """Segmented calls from two host threads, each on its own plan and stream, at the same
    time: the bucket size classes of both share the library's side streams, and every result
    must still be the oracle's (the fork and join of a call are enqueued under one lock)."""
    import threading
    import torch
    sizes = synth.segment_sizes(120, 71, 6, 18)
    offs, n = offsets_of(sizes)
    inputs = [synth.uniform_u32(n, 300 + i) for i in range(6)]
    wants = [oracle.segmented_sort(x, offs)[0] for x in inputs]
    errors = []

    def worker(tid):
        try:
            st = torch.cuda.Stream()
            plan = ds.Plan(1, False, n, max_segments=sizes.size)
            ws = plan.workspace("cuda")
            with torch.cuda.stream(st):
                to = torch.from_numpy(offs.copy()).cuda()
            for rep in range(3):
                i = 2 * rep + tid
                with torch.cuda.stream(st):
                    tk = to_dev(inputs[i])
                    plan.sort_segmented(tk, to, max_segment=int(sizes.max()), workspace=ws,
                                        stream=st)
                st.synchronize()
                if not (from_dev(tk, np.uint32) == wants[i]).all():
                    errors.append(f"thread {tid} input {i}")
        except Exception as e:  # reported below, in the test's thread
            errors.append(f"thread {tid}: {e!r}")

    say("[seg] two host threads, 3 calls each, n =", n)
    ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in ts), "a worker thread did not finish"
    assert not errors, errors
