"""dsort: deterministic sample sort for AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libdsort.so`` (C ABI in include/dsort.h).  Every step of the sort runs
in the library's HIP kernels; this module only marshals arguments.  PyTorch supplies device
memory (keys, values, workspace) and the stream.  There is no fallback: if the library is not
built, or is asked to sort host tensors, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "U32", "U64", "F32", "DsortError", "Tuning", "Plan", "load_library", "sort", "sort_pairs",
    "sort_segmented", "sort_noalloc", "Server", "SegTuning", "strerror", "EXPORTED_SYMBOLS",
    "NOALLOC_SCRATCH_BYTES",
]

U32, U64, F32 = 1, 2, 3
NOALLOC_SCRATCH_BYTES = 64 << 20  # DSORT_NOALLOC_SCRATCH_BYTES
OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP, E_CAPACITY, E_TICKET = 0, -1, -2, -3, -4, -5, -6

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsort.so")

EXPORTED_SYMBOLS = (
    "dsort_plan", "dsort_keys", "dsort_pairs", "dsort_plan_destroy", "dsort_strerror",
    "dsort_plan_geometry", "dsort_set_timing", "dsort_stage_times", "dsort_last_error",
    "dsort_segmented", "dsort_segmented_geometry",
    "dsort_server_create", "dsort_submit", "dsort_poll", "dsort_release", "dsort_server_stats",
    "dsort_server_destroy", "dsort_set_seg_tuning", "dsort_get_seg_tuning",
    "dsort_autotune_segmented", "dsort_sort_noalloc",
)


class DsortError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = f"{what}: {strerror(status)} ({status})" if what else strerror(status)
        if status == E_HIP:
            msg += f" [{load_library().dsort_last_error().decode()}]"
        super().__init__(msg)


class Tuning(ctypes.Structure):
    """dsort_tuning_t: (L, s) per level, forced level count, and ``sampling`` = 1 with ``seed``
    for the randomized-splitter comparison method (0 = Algorithm 1's chunk-end samples)."""
    _fields_ = [("sublist_len", ctypes.c_uint32), ("samples", ctypes.c_uint32),
                ("sublist_len2", ctypes.c_uint32), ("samples2", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("sampling", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


class _Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("levels", ctypes.c_uint32),
                ("sublist_len", ctypes.c_uint32), ("samples", ctypes.c_uint32),
                ("sublists", ctypes.c_uint32), ("sublist_len2", ctypes.c_uint32),
                ("samples2", ctypes.c_uint32), ("max_tiles2", ctypes.c_uint32),
                ("bucket_capacity", ctypes.c_uint32), ("bucket_bound", ctypes.c_uint32),
                ("sample_bytes", ctypes.c_uint32), ("sample_sort_global", ctypes.c_uint32),
                ("off_status", ctypes.c_uint64), ("off_samples", ctypes.c_uint64),
                ("off_sorted_samples", ctypes.c_uint64), ("off_counts", ctypes.c_uint64),
                ("off_offsets", ctypes.c_uint64), ("off_buckets", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("sampling", ctypes.c_uint32),
                ("bucket_limit", ctypes.c_uint32), ("off_overflow_count", ctypes.c_uint64),
                ("off_overflow_list", ctypes.c_uint64)]


class _SegGeometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("num_segments", ctypes.c_uint64),
                ("max_segment", ctypes.c_uint64), ("segment_limit", ctypes.c_uint64),
                ("small_capacity", ctypes.c_uint32), ("classes", ctypes.c_uint32),
                ("class_upper", ctypes.c_uint64 * 4), ("sublist_len", ctypes.c_uint32 * 4),
                ("samples", ctypes.c_uint32 * 4), ("max_long_segments", ctypes.c_uint32 * 4),
                ("max_sublists", ctypes.c_uint32 * 4), ("bucket_bound", ctypes.c_uint64 * 4),
                ("off_status", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]


class SegTuning(ctypes.Structure):
    """Long-segment classes of segmented sorts: class c holds lengths in (upper[c-1], upper[c]]
    with sublist length sublist_len[c] and samples[c] (0 = defaults); classes = 0: defaults."""
    _fields_ = [("classes", ctypes.c_uint32), ("from_cache", ctypes.c_uint32),
                ("upper", ctypes.c_uint64 * 4), ("sublist_len", ctypes.c_uint32 * 4),
                ("samples", ctypes.c_uint32 * 4)]

    def as_dict(self) -> dict:
        c = self.classes
        return {"classes": c, "upper": list(self.upper)[:c],
                "sublist_len": list(self.sublist_len)[:c], "samples": list(self.samples)[:c]}


class _Request(ctypes.Structure):
    _fields_ = [("key_type", ctypes.c_int), ("with_values", ctypes.c_int),
                ("d_keys", ctypes.c_void_p), ("d_values", ctypes.c_void_p),
                ("n", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("reserved", ctypes.c_int),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("unit", ctypes.c_uint64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "submitted", "completed", "failed", "units", "batched_units", "batched_requests",
        "max_batch", "peak_arena_bytes", "peak_running_units")]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libdsort.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdsort.so is not built ({path}); run `python -m "
                           f"paper_1002_4464_amd.build` or __graft_entry__.build()")
    # PyTorch-ROCm ships its own HIP runtime under the same soname as /opt/rocm's.  Load torch
    # first so that libdsort binds to the runtime that owns torch's device memory and streams;
    # the other order puts two HIP runtimes in one process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, U64_, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.dsort_plan.argtypes = [ctypes.POINTER(P), I, I, U64_, U64_, ctypes.POINTER(Tuning),
                               ctypes.POINTER(ctypes.c_size_t)]
    lib.dsort_plan.restype = I
    lib.dsort_keys.argtypes = [P, P, U64_, P, P]
    lib.dsort_keys.restype = I
    lib.dsort_pairs.argtypes = [P, P, P, U64_, P, P]
    lib.dsort_pairs.restype = I
    lib.dsort_plan_destroy.argtypes = [P]
    lib.dsort_plan_destroy.restype = I
    lib.dsort_strerror.argtypes = [I]
    lib.dsort_strerror.restype = ctypes.c_char_p
    lib.dsort_plan_geometry.argtypes = [P, U64_, ctypes.POINTER(_Geometry)]
    lib.dsort_plan_geometry.restype = I
    lib.dsort_set_timing.argtypes = [P, I]
    lib.dsort_set_timing.restype = I
    lib.dsort_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_uint32), I, ctypes.POINTER(I)]
    lib.dsort_stage_times.restype = I
    lib.dsort_segmented.argtypes = [P, P, P, U64_, P, U64_, U64_, P, P]
    lib.dsort_segmented.restype = I
    lib.dsort_segmented_geometry.argtypes = [P, U64_, U64_, U64_, ctypes.POINTER(_SegGeometry)]
    lib.dsort_segmented_geometry.restype = I
    lib.dsort_set_seg_tuning.argtypes = [P, ctypes.POINTER(SegTuning)]
    lib.dsort_set_seg_tuning.restype = I
    lib.dsort_get_seg_tuning.argtypes = [P, ctypes.POINTER(SegTuning)]
    lib.dsort_get_seg_tuning.restype = I
    lib.dsort_autotune_segmented.argtypes = [P, P, P, U64_, P, U64_, U64_, P, P, P, P,
                                             ctypes.c_uint32, ctypes.POINTER(SegTuning)]
    lib.dsort_autotune_segmented.restype = I
    lib.dsort_server_create.argtypes = [ctypes.POINTER(P), U64_, ctypes.c_uint32,
                                        ctypes.c_uint32]
    lib.dsort_server_create.restype = I
    lib.dsort_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(U64_)]
    lib.dsort_submit.restype = I
    lib.dsort_poll.argtypes = [P, U64_, ctypes.POINTER(_Result)]
    lib.dsort_poll.restype = I
    lib.dsort_release.argtypes = [P, U64_]
    lib.dsort_release.restype = I
    lib.dsort_server_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.dsort_server_stats.restype = I
    lib.dsort_server_destroy.argtypes = [P]
    lib.dsort_server_destroy.restype = I
    lib.dsort_sort_noalloc.argtypes = [I, I, P, P, U64_, P]
    lib.dsort_sort_noalloc.restype = I
    lib.dsort_last_error.argtypes = []
    lib.dsort_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load_library().dsort_strerror(status).decode()


def _check(rc: int, what: str):
    if rc != OK:
        raise DsortError(rc, what)


@dataclass
class Geometry:
    n: int
    levels: int
    sublist_len: int
    samples: int
    sublists: int
    sublist_len2: int
    samples2: int
    max_tiles2: int
    bucket_capacity: int
    bucket_bound: int
    sample_bytes: int
    sample_sort_global: bool
    off_status: int
    off_samples: int
    off_sorted_samples: int
    off_counts: int
    off_offsets: int
    off_buckets: int
    workspace_bytes: int
    sampling: int
    bucket_limit: int
    off_overflow_count: int
    off_overflow_list: int


@dataclass
class SegGeometry:
    n: int
    num_segments: int
    max_segment: int
    segment_limit: int
    small_capacity: int
    classes: int
    class_upper: list
    sublist_len: list
    samples: list
    max_long_segments: list
    max_sublists: list
    bucket_bound: list
    off_status: int
    workspace_bytes: int


class Plan:
    """A sort plan (host state) plus, on demand, a torch-allocated device workspace."""

    def __init__(self, key_type: int, values: bool, max_items: int, tuning: Tuning | None = None,
                 max_segments: int = 0):
        lib = load_library()
        self._lib = lib
        self.key_type = key_type
        self.values = bool(values)
        self.max_items = int(max_items)
        self.max_segments = int(max_segments)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        rc = lib.dsort_plan(ctypes.byref(h), key_type, int(self.values), self.max_items,
                            max_segments, ctypes.byref(tuning) if tuning is not None else None,
                            ctypes.byref(ws))
        _check(rc, "dsort_plan")
        self._h = h
        self.workspace_bytes = int(ws.value)
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.dsort_plan_destroy(h)
            self._h = None

    def geometry(self, n: int) -> Geometry:
        g = _Geometry()
        _check(self._lib.dsort_plan_geometry(self._h, int(n), ctypes.byref(g)),
               "dsort_plan_geometry")
        return Geometry(*[getattr(g, f) for f, _ in _Geometry._fields_])

    def segmented_geometry(self, n: int, num_segments: int, max_segment: int = 0) -> SegGeometry:
        g = _SegGeometry()
        _check(self._lib.dsort_segmented_geometry(self._h, int(n), int(num_segments),
                                                  int(max_segment), ctypes.byref(g)),
               "dsort_segmented_geometry")
        vals = []
        for f, _ in _SegGeometry._fields_:
            v = getattr(g, f)
            vals.append(list(v)[:g.classes] if isinstance(v, ctypes.Array) else v)
        return SegGeometry(*vals)

    def set_seg_tuning(self, tuning: SegTuning | None):
        _check(self._lib.dsort_set_seg_tuning(self._h, ctypes.byref(tuning) if tuning else None),
               "dsort_set_seg_tuning")

    def seg_tuning(self) -> SegTuning:
        t = SegTuning()
        _check(self._lib.dsort_get_seg_tuning(self._h, ctypes.byref(t)), "dsort_get_seg_tuning")
        return t

    def autotune_segmented(self, keys, offsets, values=None, max_segment: int = 0,
                           repeats: int = 3, workspace=None, stream=None) -> SegTuning:
        """Times candidate (L, s) per length class on this batch (left unchanged; scratch copies
        are allocated here) and installs the fastest; returns the tuning."""
        import torch
        if (values is not None) != self.values:
            raise ValueError("values must be given exactly for plans made with values")
        ksz = 8 if self.key_type == U64 else 4
        kp = self._dev_ptr(keys, ksz, "keys")
        op = self._dev_ptr(offsets, 8, "offsets")
        sk = torch.empty_like(keys)
        vp = svp = None
        sv = None
        if values is not None:
            vp = ctypes.c_void_p(self._dev_ptr(values, 4, "values"))
            sv = torch.empty_like(values)
            svp = ctypes.c_void_p(sv.data_ptr())
        ws = workspace if workspace is not None else self.workspace(keys.device, stream)
        t = SegTuning()
        rc = self._lib.dsort_autotune_segmented(
            self._h, ctypes.c_void_p(kp), vp, keys.numel(), ctypes.c_void_p(op),
            offsets.numel() - 1, int(max_segment), ctypes.c_void_p(sk.data_ptr()), svp,
            ctypes.c_void_p(ws.data_ptr()), self._stream(stream, keys.device), int(repeats),
            ctypes.byref(t))
        _check(rc, "dsort_autotune_segmented")
        del sk, sv
        return t

    def set_timing(self, enable: bool):
        """Bracket every kernel launch of later calls with HIP events (clears the record)."""
        _check(self._lib.dsort_set_timing(self._h, int(bool(enable))), "dsort_set_timing")

    def stage_times(self) -> dict:
        """{stage name: (mean ms per launch, launches)} over the recorded calls; call after
        synchronising the stream the calls ran on."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_float * cap)()
        cnt = (ctypes.c_uint32 * cap)()
        c = ctypes.c_int()
        _check(self._lib.dsort_stage_times(self._h, names, ms, cnt, cap, ctypes.byref(c)),
               "dsort_stage_times")
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(min(c.value, cap))}

    def workspace(self, device, stream=None):
        """A workspace tensor (uint8, plan.workspace_bytes) on ``device`` for calls enqueued on
        ``stream`` (default: the device's current stream), cached per (device, stream).  A
        workspace holds a call's intermediates until the call's kernels finish, so one
        workspace must never serve two streams at once; calls that pass no workspace get the
        one of their own stream."""
        import torch
        dev = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        key = (str(dev), int(stream.cuda_stream))
        ws = self._ws.get(key)
        if ws is None:
            # allocated on the stream that will use it (the caching allocator ties blocks to
            # their allocation stream)
            with torch.cuda.stream(stream):
                ws = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=dev)
            self._ws[key] = ws
        return ws

    @staticmethod
    def _dev_ptr(t, itemsize: int, what: str) -> int:
        if not t.is_cuda:
            raise ValueError(f"{what} must be a device tensor")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if t.element_size() != itemsize:
            raise ValueError(f"{what} must have {itemsize}-byte elements")
        return t.data_ptr()

    def _stream(self, stream, device):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        return ctypes.c_void_p(stream.cuda_stream)

    def sort_keys(self, keys, workspace=None, stream=None):
        """Sorts ``keys`` (a contiguous device tensor) in place; returns it."""
        if self.values:
            raise ValueError("plan was made for key/value sorts")
        ksz = 8 if self.key_type == U64 else 4
        kp = self._dev_ptr(keys, ksz, "keys")
        ws = workspace if workspace is not None else self.workspace(keys.device, stream)
        rc = self._lib.dsort_keys(self._h, ctypes.c_void_p(kp), keys.numel(),
                                  ctypes.c_void_p(ws.data_ptr()), self._stream(stream, keys.device))
        _check(rc, "dsort_keys")
        return keys

    def sort_pairs(self, keys, values, workspace=None, stream=None):
        """Stable sort of (keys, values) in place (values: 4-byte elements); returns both."""
        if not self.values:
            raise ValueError("plan was made for keys-only sorts")
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        ksz = 8 if self.key_type == U64 else 4
        kp = self._dev_ptr(keys, ksz, "keys")
        vp = self._dev_ptr(values, 4, "values")
        ws = workspace if workspace is not None else self.workspace(keys.device, stream)
        rc = self._lib.dsort_pairs(self._h, ctypes.c_void_p(kp), ctypes.c_void_p(vp),
                                   keys.numel(), ctypes.c_void_p(ws.data_ptr()),
                                   self._stream(stream, keys.device))
        _check(rc, "dsort_pairs")
        return keys, values

    def sort_segmented(self, keys, offsets, values=None, max_segment: int = 0, workspace=None,
                       stream=None):
        """Sorts every segment [offsets[g], offsets[g+1]) of ``keys`` (and ``values``) in place.
        ``offsets``: device tensor of S + 1 int64 (CSR form).  ``max_segment`` bounds the
        segment lengths (0: the longest supported).  Returns keys (and values)."""
        if (values is not None) != self.values:
            raise ValueError("values must be given exactly for plans made with values")
        ksz = 8 if self.key_type == U64 else 4
        kp = self._dev_ptr(keys, ksz, "keys")
        op = self._dev_ptr(offsets, 8, "offsets")
        if offsets.numel() < 1:
            raise ValueError("offsets needs S + 1 entries")
        vp = None
        if values is not None:
            if values.numel() != keys.numel():
                raise ValueError("keys and values differ in length")
            vp = ctypes.c_void_p(self._dev_ptr(values, 4, "values"))
        ws = workspace if workspace is not None else self.workspace(keys.device, stream)
        rc = self._lib.dsort_segmented(self._h, ctypes.c_void_p(kp), vp, keys.numel(),
                                       ctypes.c_void_p(op), offsets.numel() - 1, int(max_segment),
                                       ctypes.c_void_p(ws.data_ptr()),
                                       self._stream(stream, keys.device))
        _check(rc, "dsort_segmented")
        return keys if values is None else (keys, values)


def _key_type_of(t, key_type):
    if key_type is not None:
        return key_type
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.element_size() == 8:
        return U64
    if t.element_size() == 4:
        return U32
    raise ValueError(f"unsupported key dtype {t.dtype}")


_plans: dict = {}


def _plan_for(key_type: int, values: bool, n: int) -> Plan:
    cap = 1 << max(10, (max(n, 2) - 1).bit_length())
    k = (key_type, values, cap)
    if k not in _plans:
        _plans[k] = Plan(key_type, values, cap)
    return _plans[k]


def sort(keys, key_type: int | None = None, stream=None):
    """Sorts a contiguous device tensor in place (4-byte elements: uint32 order, or float32
    totalOrder for float32 tensors; 8-byte elements: uint64 order) and returns it.  The work is
    enqueued on ``stream`` (default: the current stream) with a workspace kept for that stream,
    so calls on different streams never share intermediates."""
    kt = _key_type_of(keys, key_type)
    return _plan_for(kt, False, keys.numel()).sort_keys(keys, stream=stream)


def sort_pairs(keys, values, key_type: int | None = None, stream=None):
    """Stable key/value sort in place; values are 4-byte elements."""
    kt = _key_type_of(keys, key_type)
    return _plan_for(kt, True, keys.numel()).sort_pairs(keys, values, stream=stream)


def sort_noalloc(keys, values=None, key_type: int | None = None, stream=None):
    """``sort`` (or ``sort_pairs`` with ``values``) through dsort_sort_noalloc: the library's
    fixed per-GPU workspace, no plan, nothing allocated.  Calls on one GPU must not overlap."""
    import torch
    kt = _key_type_of(keys, key_type)
    if not keys.is_cuda or (values is not None and not values.is_cuda):
        raise ValueError("sort_noalloc needs device tensors")
    if not keys.is_contiguous() or (values is not None and not values.is_contiguous()):
        raise ValueError("sort_noalloc needs contiguous tensors")
    if values is not None and values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    if stream is None:
        stream = torch.cuda.current_stream(keys.device)
    with torch.cuda.device(keys.device):
        rc = load_library().dsort_sort_noalloc(
            kt, int(values is not None), ctypes.c_void_p(keys.data_ptr()),
            ctypes.c_void_p(values.data_ptr()) if values is not None else None, keys.numel(),
            ctypes.c_void_p(stream.cuda_stream))
    _check(rc, "dsort_sort_noalloc")
    return keys if values is None else (keys, values)


def sort_segmented(keys, offsets, values=None, key_type: int | None = None, max_segment: int = 0,
                   stream=None):
    """Sorts each segment [offsets[g], offsets[g+1]) of a device tensor in place (key order as
    for ``sort``; with ``values``, stable as for ``sort_pairs``).  ``offsets`` is a device
    tensor of S + 1 int64 values."""
    kt = _key_type_of(keys, key_type)
    n = keys.numel()
    S = offsets.numel() - 1
    cap = 1 << max(10, (max(n, 2) - 1).bit_length())
    scap = 1 << max(6, (max(S, 1) - 1).bit_length())
    k = (kt, values is not None, cap, scap)
    if k not in _plans:
        _plans[k] = Plan(kt, values is not None, cap, max_segments=scap)
    return _plans[k].sort_segmented(keys, offsets, values, max_segment=max_segment, stream=stream)


QUEUED, RUNNING, DONE = 0, 1, 2


@dataclass
class Result:
    state: int
    t_submit_ns: int
    t_admit_ns: int
    t_done_ns: int
    unit: int

    @property
    def latency_s(self) -> float:
        return (self.t_done_ns - self.t_submit_ns) * 1e-9


class Server:
    """A served sort stream (native scheduler thread, device arena of ``budget_bytes``, ``lanes``
    HIP streams).  ``submit`` queues an in-place sort of device tensors and returns a ticket;
    the tensors are kept referenced here until the ticket is released."""

    def __init__(self, budget_bytes: int, max_inflight: int = 1024, lanes: int = 4):
        import torch  # noqa: F401  (device and runtime come from torch)
        lib = load_library()
        self._lib = lib
        h = ctypes.c_void_p()
        _check(lib.dsort_server_create(ctypes.byref(h), int(budget_bytes), int(max_inflight),
                                       int(lanes)), "dsort_server_create")
        self._h = h
        self._held = {}

    def submit(self, keys, values=None, key_type: int | None = None, sync: bool = True) -> int:
        """Queues an in-place sort.  The server's streams do not wait for other streams, so by
        default the current stream (which produced the data) is synchronised first."""
        kt = _key_type_of(keys, key_type)
        if sync:
            import torch
            torch.cuda.current_stream(keys.device).synchronize()
        ksz = 8 if kt == U64 else 4
        kp = Plan._dev_ptr(keys, ksz, "keys")
        vp = None
        if values is not None:
            if values.numel() != keys.numel():
                raise ValueError("keys and values differ in length")
            vp = Plan._dev_ptr(values, 4, "values")
        r = _Request(kt, int(values is not None), kp, vp, keys.numel())
        t = ctypes.c_uint64()
        _check(self._lib.dsort_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "dsort_submit")
        self._held[t.value] = (keys, values)
        return t.value

    def poll(self, ticket: int) -> Result:
        r = _Result()
        _check(self._lib.dsort_poll(self._h, int(ticket), ctypes.byref(r)), "dsort_poll")
        return Result(r.state, r.t_submit_ns, r.t_admit_ns, r.t_done_ns, r.unit)

    def wait(self, ticket: int, timeout_s: float = 60.0, sleep_s: float = 2e-5) -> Result:
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r.state == DONE or r.state < 0:
                if r.state < 0:
                    raise DsortError(r.state, f"request {ticket}")
                return r
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not finished after {timeout_s} s")
            time.sleep(sleep_s)

    def release(self, ticket: int):
        _check(self._lib.dsort_release(self._h, int(ticket)), "dsort_release")
        self._held.pop(ticket, None)

    def stats(self) -> dict:
        s = _ServerStats()
        _check(self._lib.dsort_server_stats(self._h, ctypes.byref(s)), "dsort_server_stats")
        return {f: int(getattr(s, f)) for f, _ in _ServerStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.dsort_server_destroy(h)
            self._h = None
            self._held.clear()

    def __del__(self):
        self.close()
