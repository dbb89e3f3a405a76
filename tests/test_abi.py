"""CPU tests of the C ABI: the library loads, exports every symbol the header declares, plans
sensible geometries, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_1002_4464_amd as ds

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "dsort.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dsort_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = ds.load_library()
    names = header_functions()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), f"{name} declared but not exported"
    assert set(names) == set(ds.EXPORTED_SYMBOLS)


def test_strerror():
    assert ds.strerror(0) == "success"
    for code in range(-6, 0):
        assert ds.strerror(code) != "unknown status"
    assert ds.strerror(12345) == "unknown status"


def test_plan_rejects_bad_arguments():
    lib = ds.load_library()
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert lib.dsort_plan(None, 1, 0, 100, 0, None, ctypes.byref(ws)) == ds.E_INVALID
    assert lib.dsort_plan(ctypes.byref(h), 1, 0, 100, 0, None, None) == ds.E_INVALID
    assert lib.dsort_plan(ctypes.byref(h), 9, 0, 100, 0, None, ctypes.byref(ws)) == ds.E_INVALID
    assert lib.dsort_plan(ctypes.byref(h), 1, 2, 100, 0, None, ctypes.byref(ws)) == ds.E_INVALID
    assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 33, 0, None,
                          ctypes.byref(ws)) == ds.E_INVALID
    # a sublist length must be a power of two or a multiple of 64 items per thread (1024 for
    # 32-bit keys), and the sample count must divide it
    for t in [(1000, 0, 0, 0, 0), (15360 + 512, 0, 0, 0, 0), (15360, 300, 0, 0, 0),
              (16384, 256, 7000, 0, 2), (16384, 256, 15360, 100, 2)]:
        bad = ds.Tuning(*t)
        assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 20, 0, ctypes.byref(bad),
                              ctypes.byref(ws)) == ds.E_UNSUPPORTED, t
    for t in [(15360, 320, 16384, 128, 2), (3072, 96, 0, 0, 0), (16384, 256, 15360, 120, 2)]:
        good = ds.Tuning(*t)
        assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 20, 0, ctypes.byref(good),
                              ctypes.byref(ws)) == ds.OK, t
        lib.dsort_plan_destroy(h)
    bad = ds.Tuning(1024, 4, 0, 0, 1)  # one level but buckets would exceed a workgroup
    assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 24, 0, ctypes.byref(bad),
                          ctypes.byref(ws)) == ds.E_UNSUPPORTED


def test_sort_rejects_bad_arguments_without_gpu():
    lib = ds.load_library()
    p = ds.Plan(ds.U32, False, 1000)
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x20000)
    # n > max_items
    assert lib.dsort_keys(p._h, fake, 1001, ws, None) == ds.E_INVALID
    # NULL keys / workspace
    assert lib.dsort_keys(p._h, None, 500, ws, None) == ds.E_INVALID
    assert lib.dsort_keys(p._h, fake, 500, None, None) == ds.E_INVALID
    # misaligned workspace and keys
    assert lib.dsort_keys(p._h, fake, 500, ctypes.c_void_p(0x20010), None) == ds.E_INVALID
    assert lib.dsort_keys(p._h, ctypes.c_void_p(0x10002), 500, ws, None) == ds.E_INVALID
    # keys-only plan used for pairs, and the reverse
    assert lib.dsort_pairs(p._h, fake, fake, 500, ws, None) == ds.E_INVALID
    q = ds.Plan(ds.U32, True, 1000)
    assert lib.dsort_keys(q._h, fake, 500, ws, None) == ds.E_INVALID
    # NULL plan
    assert lib.dsort_keys(None, fake, 500, ws, None) == ds.E_INVALID
    # n = 0 and n = 1 are no-ops that never dereference anything
    assert lib.dsort_keys(p._h, None, 0, None, None) == ds.OK
    assert lib.dsort_keys(p._h, None, 1, None, None) == ds.OK
    assert lib.dsort_plan_destroy(None) == ds.OK


def test_paper_parameter_arithmetic():
    """The paper's configuration (Section 4): n = 32M, n/m = 2K, s = 64 gives m = 16K,
    sm = 1M and the bound 2n/s = 1M; the plan reproduces it when told L and s."""
    n = 32 << 20
    p = ds.Plan(ds.U32, False, n, ds.Tuning(2048, 64, 0, 0, 0))
    g = p.geometry(n)
    assert g.sublists == 16 << 10
    assert g.sublists * g.samples == 1 << 20
    assert g.bucket_bound == 2 * n // 64 - g.sublists <= 2 * n // 64


@pytest.mark.parametrize("kt,values", [(1, False), (1, True), (2, False), (2, True), (3, False)])
def test_geometry_invariants(kt, values):
    for n in [2, 1000, 32768, 32769, 1 << 20, (1 << 20) + 3, 5_000_000, 1 << 24, 1 << 26,
              1 << 28]:
        p = ds.Plan(kt, values, n)
        g = p.geometry(n)
        assert g.workspace_bytes <= p.workspace_bytes
        if g.levels == 0:
            assert n <= g.bucket_capacity
            continue
        L, s, m = g.sublist_len, g.samples, g.sublists
        assert m == -(-n // L) and L % s == 0
        assert g.bucket_bound == 2 * m * L // s - m
        if g.levels == 1:
            assert g.bucket_bound <= g.bucket_capacity
        else:
            b1 = g.bucket_bound
            m2 = -(-b1 // g.sublist_len2)
            assert m2 * (2 * g.sublist_len2 // g.samples2 - 1) <= g.bucket_capacity
            assert g.max_tiles2 >= -(-n // g.sublist_len2) + s


def test_workspace_covers_all_smaller_sizes():
    for kt, values in [(1, False), (2, True)]:
        p = ds.Plan(kt, values, 3_000_000)
        for n in list(range(2, 70_000, 997)) + list(range(70_000, 3_000_000, 29_989)):
            assert p.geometry(n).workspace_bytes <= p.workspace_bytes


def _check_seg_geometry(g, n, S):
    """Every long class runs one level of Algorithm 1: for its longest segment (m sublists) the
    bucket bound m(2L/s - 1) fits one workgroup and the m*s samples fit the one-workgroup
    sample sort."""
    lo = g.small_capacity
    for c in range(g.classes):
        L, s, hi = g.sublist_len[c], g.samples[c], g.class_upper[c]
        assert hi > lo and L & (L - 1) == 0 and s & (s - 1) == 0
        m = -(-hi // L)
        assert g.bucket_bound[c] == m * (2 * L // s - 1) <= g.small_capacity
        assert m * s <= 16384
        assert g.max_long_segments[c] == min(S, n // (lo + 1))
        assert g.max_sublists[c] >= -(-n // L)
        lo = hi
    if g.classes:
        assert g.class_upper[-1] == g.max_segment


@pytest.mark.parametrize("kt,values", [(1, False), (1, True), (2, False), (2, True), (3, False)])
def test_segmented_geometry_invariants(kt, values):
    """Default tuning: one long class; s the smallest admissible; the plan's workspace covers
    every smaller batch."""
    n = 1 << 24
    p = ds.Plan(kt, values, n, max_segments=4096)
    lim = p.segmented_geometry(n, 4096).segment_limit
    assert lim >= 1 << 19
    for S in [1, 17, 4096]:
        for max_seg in [0, 1, 100, 8192, 8193, 16385, 32769, 100_000, lim]:
            g = p.segmented_geometry(n, S, max_seg)
            assert g.workspace_bytes <= p.workspace_bytes
            assert g.max_segment == (min(n, lim) if max_seg == 0 else max_seg)
            if g.max_segment <= g.small_capacity:
                assert g.classes == 0
                continue
            assert g.classes == 1
            _check_seg_geometry(g, n, S)
            L, s = g.sublist_len[0], g.samples[0]
            m = -(-g.max_segment // L)
            assert s == 1 or m * (2 * L // (s // 2) - 1) > g.small_capacity
    with pytest.raises(ds.DsortError) as e:
        p.segmented_geometry(n, 10, lim + 1)
    assert e.value.status == ds.E_UNSUPPORTED
    with pytest.raises(ds.DsortError) as e:
        p.segmented_geometry(n, 4097, 0)
    assert e.value.status == ds.E_INVALID


def _tuning(classes, upper, L, s):
    t = ds.SegTuning()
    t.classes = classes
    for i in range(classes):
        t.upper[i], t.sublist_len[i], t.samples[i] = upper[i], L[i], s[i]
    return t


@pytest.mark.parametrize("kt,values", [(1, False), (1, True), (2, True), (3, False)])
def test_segmented_tuning_classes(kt, values):
    """Tunings the autotuner can pick fit the plan's workspace; the geometry follows them."""
    n = 1 << 24
    p = ds.Plan(kt, values, n, max_segments=4096)
    lim = p.segmented_geometry(n, 4096).segment_limit
    cap = p.segmented_geometry(n, 4096).small_capacity
    upper = [cap * 4, cap * 16, cap * 64, 1 << 62]
    for L in (2048, 4096, 8192):
        for mult in (1, 2):
            t = _tuning(4, upper, [L, L, 0, 0], [0, 0, 0, 0])
            p.set_seg_tuning(t)
            g = p.segmented_geometry(n, 4096, lim)
            assert g.workspace_bytes <= p.workspace_bytes
            _check_seg_geometry(g, n, 4096)
            assert g.sublist_len[0] == L
    p.set_seg_tuning(None)
    assert p.seg_tuning().classes == 0
    # infeasible or malformed tunings are refused and leave the tuning unchanged
    with pytest.raises(ds.DsortError) as e:
        p.set_seg_tuning(_tuning(2, [cap * 4, cap * 2], [0, 0], [0, 0]))
    assert e.value.status == ds.E_INVALID
    with pytest.raises(ds.DsortError) as e:
        p.set_seg_tuning(_tuning(1, [1 << 62], [3000], [0]))
    assert e.value.status == ds.E_UNSUPPORTED
    with pytest.raises(ds.DsortError) as e:
        p.set_seg_tuning(_tuning(1, [1 << 62], [0], [3]))  # s not a power of two
    assert e.value.status == ds.E_UNSUPPORTED
    assert p.seg_tuning().classes == 0
    # an (L, s) that cannot bound a call's buckets falls back to the defaults for that call
    p.set_seg_tuning(_tuning(2, [cap * 4, 1 << 62], [2048, 2048], [1, 1]))
    g = p.segmented_geometry(n, 4096, lim)
    _check_seg_geometry(g, n, 4096)
    default = ds.Plan(kt, values, n, max_segments=4096).segmented_geometry(n, 4096, lim)
    assert g.samples[-1] == default.samples[0] and g.sublist_len[-1] == default.sublist_len[0]


def test_segmented_rejects_bad_arguments_without_gpu():
    lib = ds.load_library()
    p = ds.Plan(ds.U32, False, 1000, max_segments=8)
    fake = ctypes.c_void_p(0x10000)
    offs = ctypes.c_void_p(0x30000)
    ws = ctypes.c_void_p(0x20000)
    seg = lib.dsort_segmented
    assert seg(p._h, fake, None, 1001, offs, 8, 0, ws, None) == ds.E_INVALID  # n too large
    assert seg(p._h, fake, None, 1000, offs, 9, 0, ws, None) == ds.E_INVALID  # S too large
    assert seg(p._h, fake, fake, 1000, offs, 8, 0, ws, None) == ds.E_INVALID  # values, no plan
    assert seg(p._h, None, None, 1000, offs, 8, 0, ws, None) == ds.E_INVALID
    assert seg(p._h, fake, None, 1000, None, 8, 0, ws, None) == ds.E_INVALID
    assert seg(p._h, fake, None, 1000, ctypes.c_void_p(0x30004), 8, 0, ws, None) == ds.E_INVALID
    assert seg(p._h, fake, None, 1000, offs, 8, 0, ctypes.c_void_p(0x20040), None) == ds.E_INVALID
    assert seg(None, fake, None, 1000, offs, 8, 0, ws, None) == ds.E_INVALID
    q = ds.Plan(ds.U32, True, 1000, max_segments=8)
    assert seg(q._h, fake, None, 1000, offs, 8, 0, ws, None) == ds.E_INVALID  # values missing
    # empty batch / empty array: no-ops that touch nothing
    assert seg(p._h, None, None, 0, None, 8, 0, None, None) == ds.OK
    assert seg(p._h, None, None, 1000, None, 0, 0, None, None) == ds.OK
    # a plan without segments accepts none
    r = ds.Plan(ds.U32, False, 1000)
    assert seg(r._h, fake, None, 1000, offs, 1, 0, ws, None) == ds.E_INVALID


def test_server_rejects_bad_arguments_without_gpu():
    lib = ds.load_library()
    h = ctypes.c_void_p()
    assert lib.dsort_server_create(None, 1 << 30, 16, 2) == ds.E_INVALID
    assert lib.dsort_server_create(ctypes.byref(h), 1000, 16, 2) == ds.E_INVALID  # < 1 MiB
    assert lib.dsort_server_create(ctypes.byref(h), 1 << 30, 0, 2) == ds.E_INVALID
    assert lib.dsort_server_create(ctypes.byref(h), 1 << 30, 16, 0) == ds.E_INVALID
    assert lib.dsort_server_create(ctypes.byref(h), 1 << 30, 16, 17) == ds.E_INVALID
    t = ctypes.c_uint64()
    r = ds._Request(1, 0, None, None, 10)
    assert lib.dsort_submit(None, ctypes.byref(r), ctypes.byref(t)) == ds.E_INVALID
    res = ds._Result()
    assert lib.dsort_poll(None, 1, ctypes.byref(res)) == ds.E_INVALID
    assert lib.dsort_release(None, 1) == ds.E_INVALID
    st = ds._ServerStats()
    assert lib.dsort_server_stats(None, ctypes.byref(st)) == ds.E_INVALID
    assert lib.dsort_server_destroy(None) == ds.OK


def test_largest_plannable_sizes():
    """Two levels of Algorithm 1 reach about 2^30 32-bit keys (less for wider items); a plan
    for more is refused up front (DSORT_E_UNSUPPORTED), never at sort time."""
    def ok(kt, v, n):
        try:
            ds.Plan(kt, v, n)
            return True
        except ds.DsortError as e:
            assert e.status == ds.E_UNSUPPORTED
            return False
    for kt, v, limit in [(1, False, 1108377600), (3, False, 1108377600), (1, True, 554188800),
                         (2, False, 554188800), (2, True, 286326784)]:
        assert ok(kt, v, limit) and not ok(kt, v, limit + 1)


NOALLOC_LIMITS = [(ds.U32, 0, 13_801_792), (ds.F32, 0, 13_801_792), (ds.U32, 1, 7_615_552),
                  (ds.U64, 0, 7_086_432), (ds.U64, 1, 4_755_104)]


@pytest.mark.parametrize("kt,values,limit", NOALLOC_LIMITS)
def test_noalloc_limits_without_gpu(kt, values, limit):
    """dsort_sort_noalloc serves n up to the stated limits (the automatic plan's workspace fits
    the fixed array) and refuses one more item with DSORT_E_CAPACITY before touching the GPU;
    bad arguments are refused the same way."""
    lib = ds.load_library()
    p = ds.Plan(kt, bool(values), limit + 1)
    assert p.geometry(limit).workspace_bytes <= ds.NOALLOC_SCRATCH_BYTES
    assert p.geometry(limit + 1).workspace_bytes > ds.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x10000)
    fv = fake if values else None
    assert lib.dsort_sort_noalloc(kt, values, fake, fv, limit + 1, None) == ds.E_CAPACITY
    assert lib.dsort_sort_noalloc(kt, values, None, fv, 1000, None) == ds.E_INVALID
    assert lib.dsort_sort_noalloc(kt, values, ctypes.c_void_p(0x10002), fv, 1000,
                                  None) == ds.E_INVALID
    assert lib.dsort_sort_noalloc(kt, 1, fake, None, 1000, None) == ds.E_INVALID
    assert lib.dsort_sort_noalloc(kt, 0, fake, fake, 1000, None) == ds.E_INVALID
    assert lib.dsort_sort_noalloc(7, values, fake, fv, 1000, None) == ds.E_INVALID
    assert lib.dsort_sort_noalloc(kt, values, None, None, 1, None) == ds.OK


def _random_tuning(**kw):
    t = ds.Tuning(kw.get("L", 0), kw.get("s", 0), kw.get("L2", 0), kw.get("s2", 0),
                  kw.get("levels", 0))
    t.sampling = kw.get("sampling", 1)
    t.seed = kw.get("seed", 1)
    return t


def test_random_sampling_plans_without_gpu():
    """Randomized-sample plans: same level structure as the deterministic plan, a bucket limit
    for the normal path (one workgroup at one level; the second level's capacity at two), a
    workspace that also holds the deterministic plan's further runs, and refusal of segmented
    calls and of unknown sampling modes."""
    lib = ds.load_library()
    for n, kt, vals in [(1_000_003, ds.U32, False), (1 << 24, ds.U32, False),
                        (300_001, ds.U64, True), (1 << 26, ds.U32, True)]:
        det = ds.Plan(kt, vals, n)
        rnd = ds.Plan(kt, vals, n, _random_tuning(seed=5))
        gd, gr = det.geometry(n), rnd.geometry(n)
        assert (gr.levels, gr.sublist_len, gr.samples, gr.sublist_len2, gr.samples2) == \
            (gd.levels, gd.sublist_len, gd.samples, gd.sublist_len2, gd.samples2)
        assert gd.sampling == 0 and gd.bucket_limit == 0 and gr.sampling == 1
        if gr.levels == 1:
            assert gr.bucket_limit == gr.bucket_capacity
        else:
            # at least the deterministic bound, and a whole number of level-2 sublists
            assert gr.bucket_limit >= gd.bucket_bound
            assert gr.bucket_limit % gr.sublist_len2 == 0
        assert gr.off_overflow_list > 0 and gr.off_overflow_count > gr.off_status
        assert rnd.workspace_bytes >= det.workspace_bytes
    h = ctypes.c_void_p()
    wsb = ctypes.c_size_t()
    bad = _random_tuning(sampling=2)
    assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 20, 0, ctypes.byref(bad),
                          ctypes.byref(wsb)) == ds.E_UNSUPPORTED
    p = ds.Plan(ds.U32, False, 1 << 20, _random_tuning(), max_segments=16)
    fake = ctypes.c_void_p(0x10000)
    assert lib.dsort_segmented(p._h, fake, None, 1000, fake, 4, 0, ctypes.c_void_p(0x20000),
                               None) == ds.E_UNSUPPORTED
