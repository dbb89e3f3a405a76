"""GPU: dsort_sort_noalloc (the library's fixed per-GPU workspace, nothing allocated) gives
bit-identical results to dsort_keys / dsort_pairs with a caller workspace, on two calls in a
row whose second input is smaller (the array keeps the first call's intermediates)."""
import ctypes

import numpy as np
import pytest

import synth
from helpers import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

# Largest n per layout whose automatic-plan workspace fits the 64 MiB array.
LIMITS = {("u32", False): 13_801_792, ("u32", True): 7_615_552, ("u64", False): 7_086_432,
          ("u64", True): 4_755_104}


@pytest.fixture(scope="module")
def ds():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1002_4464_amd as d
    d.load_library()
    return d


def _keys(kind, n, seed):
    if kind == "u32":
        return synth.uniform_u32(n, seed)
    if kind == "f32":
        return synth.normal_f32_segments([n], seed)
    return synth.zipf_u64(n, seed, distinct=1 << 12)


def _noalloc(ds, kt, tk, tv):
    import torch
    lib = ds.load_library()
    st = torch.cuda.current_stream()
    rc = lib.dsort_sort_noalloc(kt, int(tv is not None), ctypes.c_void_p(tk.data_ptr()),
                                ctypes.c_void_p(tv.data_ptr()) if tv is not None else None,
                                tk.numel(), ctypes.c_void_p(st.cuda_stream))
    assert rc == ds.OK, ds.strerror(rc)


def _with_plan(ds, kt, keys, vals):
    import torch
    plan = ds.Plan(kt, vals is not None, keys.size)
    tk = to_dev(keys)
    if vals is None:
        plan.sort_keys(tk)
        tv = None
    else:
        tv = to_dev(vals)
        plan.sort_pairs(tk, tv)
    torch.cuda.synchronize()
    return from_dev(tk, keys.dtype), (from_dev(tv, np.uint32) if tv is not None else None)


@pytest.mark.parametrize("kind,pairs,sizes", [
    ("u32", False, [LIMITS[("u32", False)], 300_007]),   # two levels, then one
    ("f32", False, [4_000_003, 40_000]),                  # one level, then one tile
    ("u32", True, [LIMITS[("u32", True)], 1_000_001]),
    ("u64", False, [6_000_000, 123_457]),
    ("u64", True, [LIMITS[("u64", True)], 20_001]),
])
def test_noalloc_matches_plan_entry_point(ds, kind, pairs, sizes):
    import torch
    kt = {"u32": ds.U32, "f32": ds.F32, "u64": ds.U64}[kind]
    for call, n in enumerate(sizes):
        say(f"noalloc {kind} pairs={pairs} call {call} n={n}")
        keys = _keys(kind, n, 700 + 10 * call + len(kind))
        vals = synth.index_values(n) if pairs else None
        want_k, want_v = _with_plan(ds, kt, keys, vals)
        tk = to_dev(keys)
        tv = to_dev(vals) if pairs else None
        _noalloc(ds, kt, tk, tv)
        torch.cuda.synchronize()
        got_k = from_dev(tk, keys.dtype)
        assert (got_k.view(np.uint8) == want_k.view(np.uint8)).all(), f"keys differ, call {call}"
        if pairs:
            assert (from_dev(tv, np.uint32) == want_v).all(), f"values differ, call {call}"


def test_noalloc_rejects_beyond_limit(ds):
    """One item past the limit is refused before anything is enqueued; the tensors stay as
    they were."""
    import torch
    lib = ds.load_library()
    n = LIMITS[("u64", True)] + 1
    keys = _keys("u64", n, 99)
    tk = to_dev(keys)
    tv = to_dev(synth.index_values(n))
    st = torch.cuda.current_stream()
    rc = lib.dsort_sort_noalloc(ds.U64, 1, ctypes.c_void_p(tk.data_ptr()),
                                ctypes.c_void_p(tv.data_ptr()), n, ctypes.c_void_p(st.cuda_stream))
    assert rc == ds.E_CAPACITY
    torch.cuda.synchronize()
    assert (from_dev(tk, np.uint64) == keys).all()
