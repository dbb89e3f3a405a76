"""CPU oracle for the deterministic sample sort (Algorithm 1, Section 4 of the paper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does.  The arithmetic lives in ``dss_oracle.c``
(plain single-threaded C); this module only compiles it with gcc and marshals numpy arrays.
It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dss_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U32, U64, F32 = 1, 2, 3
_KIND = {np.dtype(np.uint32): U32, np.dtype(np.uint64): U64, np.dtype(np.float32): F32}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single-threaded) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Trace(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "sample_key", "sample_pos", "splitter_key", "splitter_pos", "count", "offset",
        "bucket_size", "reloc_key", "reloc_val")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        # DSS_ORACLE_LIB: a deliberately broken build, used only by the mutation tests to show
        # that the pins catch planted mistakes.
        path = os.environ.get("DSS_ORACLE_LIB")
        if not path:
            build(force=False)
            path = _LIB
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_dss.argtypes = [ctypes.c_int, P, P, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_uint64, P, P, ctypes.POINTER(_Trace)]
        lib.oracle_dss.restype = ctypes.c_int
        lib.oracle_dss_sampled.argtypes = [ctypes.c_int, P, P, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, P, P,
                                           ctypes.POINTER(_Trace)]
        lib.oracle_dss_sampled.restype = ctypes.c_int
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_stable_sort.argtypes = [ctypes.c_int, P, P, ctypes.c_uint64, P, P]
        lib.oracle_stable_sort.restype = ctypes.c_int
        lib.oracle_f32_order.argtypes = [ctypes.c_uint32]
        lib.oracle_f32_order.restype = ctypes.c_uint32
        lib.oracle_f32_unorder.argtypes = [ctypes.c_uint32]
        lib.oracle_f32_unorder.restype = ctypes.c_uint32
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _kind(keys: np.ndarray) -> int:
    try:
        return _KIND[keys.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {keys.dtype}") from None


@dataclass
class Trace:
    """Intermediates of Algorithm 1 at one (L, s).  Rows of ``count``/``offset`` are sublists."""
    n: int
    L: int
    s: int
    m: int
    sample_key: np.ndarray
    sample_pos: np.ndarray
    splitter_key: np.ndarray
    splitter_pos: np.ndarray
    count: np.ndarray
    offset: np.ndarray
    bucket_size: np.ndarray
    reloc_key: np.ndarray
    reloc_val: np.ndarray


def dss(keys: np.ndarray, L: int, s: int, values: np.ndarray | None = None,
        trace: bool = False, reloc: bool = True, sampling: int = 0, seed: int = 0):
    """Algorithm 1 on ``keys`` (uint32, uint64 or float32) with sublist length L, s samples.

    Returns ``(sorted_keys, sorted_values_or_None, Trace_or_None)``.  With ``reloc=False`` the
    trace leaves out the array after Step 8 (``reloc_key``/``reloc_val`` are None), which at
    large n is the bulk of its memory.  ``sampling=1`` takes Step 3's samples at random
    positions drawn from ``seed`` (the randomized-splitter variant, reading R8 of the C source).
    """
    lib = _load()
    keys = np.ascontiguousarray(keys)
    kind = _kind(keys)
    n = int(keys.size)
    if values is not None:
        values = np.ascontiguousarray(values, dtype=np.uint32)
        assert values.size == n
    out_k = np.empty_like(keys)
    out_v = np.empty(n, dtype=np.uint32) if values is not None else None
    tr_obj = None
    tr_ptr = None
    if trace and n > 0:
        m = -(-n // L)
        u64 = np.uint64
        tr_obj = Trace(n, L, s, m,
                       np.empty(m * s, u64), np.empty(m * s, u64), np.empty(s, u64),
                       np.empty(s, u64), np.empty((m, s), u64), np.empty((m, s), u64),
                       np.empty(s, u64), np.empty(m * L, keys.dtype) if reloc else None,
                       np.empty(m * L, np.uint32) if reloc else None)
        tr_ptr = ctypes.pointer(_Trace(*[_ptr(getattr(tr_obj, f)) for f, _ in _Trace._fields_]))
    rc = lib.oracle_dss_sampled(kind, _ptr(keys), _ptr(values), n, L, s, int(sampling),
                                int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out_k), _ptr(out_v), tr_ptr)
    if rc != 0:
        raise ValueError(f"oracle_dss failed with status {rc} (n={n}, L={L}, s={s}, "
                         f"sampling={sampling})")
    return out_k, out_v, tr_obj


def stable_sort(keys: np.ndarray, values: np.ndarray | None = None):
    """The plain definition of the result: stable sort by key order."""
    lib = _load()
    keys = np.ascontiguousarray(keys)
    kind = _kind(keys)
    n = int(keys.size)
    if values is not None:
        values = np.ascontiguousarray(values, dtype=np.uint32)
    out_k = np.empty_like(keys)
    out_v = np.empty(n, dtype=np.uint32) if values is not None else None
    rc = lib.oracle_stable_sort(kind, _ptr(keys), _ptr(values), n, _ptr(out_k), _ptr(out_v))
    if rc != 0:
        raise ValueError(f"oracle_stable_sort failed with status {rc}")
    return out_k, out_v


def segmented_sort(keys: np.ndarray, offsets, values: np.ndarray | None = None):
    """A batch of independent sorts: segment g, the range [offsets[g], offsets[g+1]), is sorted
    on its own by the plain definition (stable sort by key order, Algorithm 1's output applied
    per segment); items outside every segment keep their places.  Offsets must be
    non-decreasing and within the array."""
    offsets = [int(x) for x in offsets]
    out_k = np.array(keys, copy=True)
    out_v = np.array(values, dtype=np.uint32, copy=True) if values is not None else None
    for lo, hi in zip(offsets[:-1], offsets[1:]):
        if not 0 <= lo <= hi <= keys.size:
            raise ValueError(f"bad segment [{lo}, {hi})")
        if hi - lo < 2:
            continue
        k, v = stable_sort(keys[lo:hi], None if values is None else values[lo:hi])
        out_k[lo:hi] = k
        if values is not None:
            out_v[lo:hi] = v
    return out_k, out_v


def splitmix64(seed: int, c: int) -> int:
    """Draw ``c`` of the oracle's own SplitMix64 stream seeded with ``seed`` (reading R8)."""
    return int(_load().oracle_splitmix64(int(seed) & 0xFFFFFFFFFFFFFFFF, int(c)))


def f32_order(bits: int) -> int:
    """totalOrder image of one binary32 bit pattern."""
    return int(_load().oracle_f32_order(bits))


def f32_unorder(image: int) -> int:
    return int(_load().oracle_f32_unorder(image))
