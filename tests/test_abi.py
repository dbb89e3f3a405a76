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
    bad = ds.Tuning(1000, 0, 0, 0, 0)  # not a power of two
    assert lib.dsort_plan(ctypes.byref(h), 1, 0, 1 << 20, 0, ctypes.byref(bad),
                          ctypes.byref(ws)) == ds.E_UNSUPPORTED
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
