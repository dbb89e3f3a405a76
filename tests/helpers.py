"""Shared test helpers: moving numpy arrays to and from the GPU, reading the workspace, and
running independent oracle calls on several host threads (the oracle is single-threaded C
called through ctypes, which releases the GIL, so independent calls run side by side)."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

# Host threads for oracle work (a GPU machine gives one GPU 16 host cores).
ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))
_pool = None


def oracle_pool() -> ThreadPoolExecutor:
    """Process-wide thread pool for oracle calls that run beside GPU work."""
    global _pool
    if _pool is None:
        _pool = ThreadPoolExecutor(max_workers=ORACLE_THREADS)
    return _pool


def oracle_segmented(keys: np.ndarray, offsets, values=None, threads: int = ORACLE_THREADS):
    """``oracle.segmented_sort`` computed with segments spread over ``threads`` host threads
    (each thread runs the oracle's stable sort on its own segments, in place of one loop)."""
    import oracle
    offsets = [int(x) for x in offsets]
    out_k = np.array(keys, copy=True)
    out_v = np.array(values, dtype=np.uint32, copy=True) if values is not None else None
    segs = [(lo, hi) for lo, hi in zip(offsets[:-1], offsets[1:]) if hi - lo >= 2]
    for lo, hi in segs:
        if not 0 <= lo <= hi <= keys.size:
            raise ValueError(f"bad segment [{lo}, {hi})")

    def run(part):
        for lo, hi in part:
            k, v = oracle.stable_sort(keys[lo:hi], None if values is None else values[lo:hi])
            out_k[lo:hi] = k
            if values is not None:
                out_v[lo:hi] = v

    # deal segments round-robin by size so every thread gets a similar share
    order = sorted(segs, key=lambda r: r[0] - r[1])
    parts = [order[i::threads] for i in range(threads)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for f in [ex.submit(run, part) for part in parts if part]:
            f.result()
    return out_k, out_v

_VIEW = {np.dtype(np.uint32): np.int32, np.dtype(np.float32): np.int32,
         np.dtype(np.uint64): np.int64}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(_VIEW[a.dtype]).copy()).cuda()


def from_dev(t, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


def ws_view(ws, offset: int, count: int, dtype) -> np.ndarray:
    """``count`` items of ``dtype`` at byte ``offset`` of a workspace tensor."""
    nbytes = count * np.dtype(dtype).itemsize
    return ws[offset:offset + nbytes].cpu().numpy().view(dtype)


def samples_from_ws(ws, offset: int, count: int, sample_bytes: int):
    """Decodes sample composites into (key, pos) uint64 arrays."""
    if sample_bytes == 8:
        c = ws_view(ws, offset, count, np.uint64)
        return c >> np.uint64(32), c & np.uint64(0xFFFFFFFF)
    raw = ws_view(ws, offset, count * 2, np.uint64).reshape(count, 2)
    return raw[:, 0].copy(), raw[:, 1] & np.uint64(0xFFFFFFFF)


KT = {np.dtype(np.uint32): 1, np.dtype(np.uint64): 2, np.dtype(np.float32): 3}


def gpu_sort(ds, keys, values=None, tuning=None, plan=None):
    import torch
    kt = KT[keys.dtype]
    if plan is None:
        plan = ds.Plan(kt, values is not None, max(keys.size, 2), tuning)
    tk = to_dev(keys)
    ws = plan.workspace(tk.device)
    if values is None:
        plan.sort_keys(tk, ws)
        tv = None
    else:
        tv = to_dev(values)
        plan.sort_pairs(tk, tv, ws)
    torch.cuda.synchronize()
    geo = plan.geometry(keys.size)
    status = int(ws_view(ws, geo.off_status, 1, np.uint32)[0])
    assert status == 0, f"kernel status flags {status:#x}"
    out_k = from_dev(tk, keys.dtype)
    out_v = from_dev(tv, np.uint32) if tv is not None else None
    return out_k, out_v, geo, ws


def check_level1(geo, ws, tr, n):
    """Level-1 intermediates equal the oracle's at the same (L, s)."""
    m, s = geo.sublists, geo.samples
    assert (m, s, geo.sublist_len) == (tr.m, tr.s, tr.L)
    sk, sp = samples_from_ws(ws, geo.off_sorted_samples, m * s, geo.sample_bytes)
    assert (sk == tr.sample_key).all(), "sorted sample keys (Step 4)"
    assert (sp == tr.sample_pos).all(), "sorted sample positions (Step 4)"
    counts = ws_view(ws, geo.off_counts, m * s, np.uint32).reshape(m, s)
    assert (counts == tr.count).all(), "a_ij (Step 6)"
    offs = ws_view(ws, geo.off_offsets, m * s, np.uint32).reshape(m, s)
    assert (offs == tr.offset).all(), "l_ij (Step 7)"
    b = ws_view(ws, geo.off_buckets, 4 * s, np.uint32).reshape(s, 4).astype(np.int64)
    begin = tr.offset[0].astype(np.int64)
    real = np.clip(n - begin, 0, tr.bucket_size.astype(np.int64))
    assert (b[:, 0] == begin).all(), "bucket starts (Step 8)"
    assert (b[:, 1] == real).all(), "bucket sizes (Step 8)"
    assert (b[:, 2] == np.arange(s) * m).all() and (b[:, 3] == m).all(), "bucket piece ranges"
