"""Shared test helpers: moving numpy arrays to and from the GPU, and reading the workspace."""
import sys

import numpy as np

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
