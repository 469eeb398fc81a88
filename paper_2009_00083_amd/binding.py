"""ctypes binding of libpcrit.so (argument marshalling only).

Every function forwards to the C ABI declared in ``include/pcrit.h``; the
classification itself runs in the library's HIP kernels.  Device buffers are
torch tensors on a ROCm device; the stream is torch's current stream unless
one is given.  A missing library raises ``PcritError`` -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import functools
import os
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

E_ARG, E_DIMS, E_LEVEL, E_CAPACITY, E_NAN, E_HIP, E_OOM = -1, -2, -3, -4, -5, -6, -7
E_SCRATCH = -8
NOALLOC_SCRATCH_BYTES = 32 << 20

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpcrit.so")
_lib = None

EXPORTED = ("pcrit_create", "pcrit_destroy", "pcrit_strerror",
            "pcrit_max_level", "pcrit_level_dims", "pcrit_link_table",
            "pcrit_classify", "pcrit_classify_noalloc", "pcrit_progressive",
            "pcrit_progressive_async",
            "pcrit_set_kernel_timing", "pcrit_kernel_ms", "pcrit_preview_f1",
            "pcrit_preview_f1_levels", "pcrit_mlp_feature_level", "pcrit_mlp_features",
            "pcrit_mlp_labels", "pcrit_mlp_forward", "pcrit_mlp_backward",
            "pcrit_mlp_adam", "pcrit_region_count", "pcrit_progressive_timeline",
            "pcrit_classify_batch", "pcrit_order_field", "pcrit_extrema",
            "pcrit_lts_propagate", "pcrit_lts_merged", "pcrit_set_batch_config",
            "pcrit_get_batch_config", "pcrit_batch_autotune")
MLP_PARAMS = 6337
MLP_INPUTS = 32


class PcritError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _strerror(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise PcritError(E_HIP, f"{_LIB_PATH} is not built "
                                "(run __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    p64 = ctypes.POINTER(i64)
    lib.pcrit_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.pcrit_create.restype = i32
    lib.pcrit_destroy.argtypes = [vp]
    lib.pcrit_destroy.restype = None
    lib.pcrit_strerror.argtypes = [i32]
    lib.pcrit_strerror.restype = ctypes.c_char_p
    lib.pcrit_max_level.argtypes = [i64, i64, i64, ctypes.POINTER(i32)]
    lib.pcrit_max_level.restype = i32
    lib.pcrit_level_dims.argtypes = [i64, i64, i64, i32, vp]
    lib.pcrit_level_dims.restype = i32
    lib.pcrit_link_table.argtypes = [i32, vp, i64]
    lib.pcrit_link_table.restype = i32
    lib.pcrit_classify.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp, vp, vp,
                                   i64, p64, vp]
    lib.pcrit_classify.restype = i32
    lib.pcrit_classify_noalloc.argtypes = lib.pcrit_classify.argtypes
    lib.pcrit_classify_noalloc.restype = i32
    lib.pcrit_classify_batch.argtypes = [vp, vp, i32, vp, vp, vp, i64, vp, vp]
    lib.pcrit_classify_batch.restype = i32
    lib.pcrit_order_field.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp]
    lib.pcrit_order_field.restype = i32
    lib.pcrit_extrema.argtypes = [vp, vp, vp, i64, i64, i64, vp, i64, vp]
    lib.pcrit_extrema.restype = i32
    lib.pcrit_lts_propagate.argtypes = [vp, vp, vp, vp, i64, i64, i64, vp, i64, i32,
                                        ctypes.c_float, i32, i32, vp, vp, vp]
    lib.pcrit_lts_propagate.restype = i32
    lib.pcrit_lts_merged.argtypes = [vp, vp, vp, vp, i64, i64, i64, vp, i64, i32,
                                     ctypes.c_float, i32, i32, vp, vp, vp]
    lib.pcrit_lts_merged.restype = i32
    lib.LEVEL_CB = ctypes.CFUNCTYPE(None, i32, i64, vp)
    lib.NULL_CB = ctypes.cast(None, lib.LEVEL_CB)
    lib.pcrit_progressive.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, vp,
                                      i64, vp, vp, vp, lib.LEVEL_CB, vp]
    lib.pcrit_progressive.restype = i32
    lib.pcrit_progressive_async.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, i64, vp]
    lib.pcrit_progressive_async.restype = i32
    lib.pcrit_set_kernel_timing.argtypes = [vp, ctypes.c_uint64]
    lib.pcrit_set_kernel_timing.restype = i32
    lib.pcrit_set_batch_config.argtypes = [vp, i32, i64]
    lib.pcrit_set_batch_config.restype = i32
    lib.pcrit_get_batch_config.argtypes = [vp, vp, vp]
    lib.pcrit_get_batch_config.restype = i32
    lib.pcrit_batch_autotune.argtypes = [vp, vp, i32, vp, vp, vp, i64, i32, vp, vp, vp]
    lib.pcrit_batch_autotune.restype = i32
    lib.pcrit_kernel_ms.argtypes = [vp, vp, vp, i32]
    lib.pcrit_kernel_ms.restype = i32
    lib.pcrit_preview_f1.argtypes = [i64, i64, i64, i32, vp, vp, i64, vp, vp,
                                     i64, ctypes.POINTER(ctypes.c_double), p64]
    lib.pcrit_preview_f1.restype = i32
    lib.pcrit_preview_f1_levels.argtypes = [i64, i64, i64, vp, vp, vp, i64, vp, vp, i64,
                                            ctypes.POINTER(ctypes.c_double), p64]
    lib.pcrit_preview_f1_levels.restype = i32
    lib.pcrit_mlp_feature_level.argtypes = [i64, i64, i64, ctypes.POINTER(i32)]
    lib.pcrit_mlp_feature_level.restype = i32
    lib.pcrit_mlp_features.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp]
    lib.pcrit_mlp_features.restype = i32
    lib.pcrit_mlp_labels.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp]
    lib.pcrit_mlp_labels.restype = i32
    lib.pcrit_mlp_forward.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.pcrit_mlp_forward.restype = i32
    lib.pcrit_mlp_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
    lib.pcrit_mlp_backward.restype = i32
    lib.pcrit_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_float, i32]
    lib.pcrit_mlp_adam.restype = i32
    lib.pcrit_region_count.argtypes = [i64, i64, i64, i32, ctypes.POINTER(i32)]
    lib.pcrit_region_count.restype = i32
    lib.pcrit_progressive_timeline.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, i64, i32,
                                               i32, vp, vp, vp, vp, vp]
    lib.pcrit_progressive_timeline.restype = i32
    _lib = lib
    return lib


def _strerror(status: int) -> str:
    try:
        return _load().pcrit_strerror(status).decode()
    except PcritError:
        return f"status {status}"


def _check(status: int, what: str):
    if status != 0:
        raise PcritError(status, what)


def _shape3(shape):
    shape = tuple(int(s) for s in shape)
    if len(shape) == 3:
        nz, ny, nx = shape
    elif len(shape) == 2:
        (ny, nx), nz = shape, 1
    else:
        raise PcritError(E_DIMS, "field must be (nz, ny, nx) or (ny, nx)")
    return nx, ny, nz


def max_level(shape) -> int:
    k = ctypes.c_int(0)
    nx, ny, nz = _shape3(shape)
    _check(_load().pcrit_max_level(nx, ny, nz, ctypes.byref(k)), "max_level")
    return k.value


def level_dims(shape, level: int):
    """(n_x, n_y, n_z) samples of level `level`."""
    m = np.zeros(3, np.int64)
    nx, ny, nz = _shape3(shape)
    _check(_load().pcrit_level_dims(nx, ny, nz, level, m.ctypes.data),
           "level_dims")
    return tuple(int(v) for v in m)


@functools.lru_cache(maxsize=64)
def _hierarchy(shape):
    """(k_max, vertices of all levels) of a grid shape (cached: the
    progressive call is issued per step)."""
    kmax = max_level(shape)
    total = 0
    for k in range(kmax + 1):
        m = level_dims(shape, k)
        total += m[0] * m[1] * m[2]
    return kmax, total


def link_table(dim: int) -> np.ndarray:
    """The host-built link-pattern table the kernels use (16384 or 64 B)."""
    n = 1 << 14 if dim == 3 else 1 << 6
    t = np.zeros(n, np.uint8)
    _check(_load().pcrit_link_table(dim, t.ctypes.data, n), "link_table")
    return t


class Context:
    """Owns the device lookup tables, scratch and events of one device."""

    def __init__(self, device: int = 0):
        lib = _load()
        self._ptr = ctypes.c_void_p()
        _check(lib.pcrit_create(ctypes.byref(self._ptr), int(device)),
               "pcrit_create")
        self.device = int(device)

    @property
    def handle(self):
        return self._ptr

    def close(self):
        if self._ptr:
            _load().pcrit_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_batch_config(self, group: int = 0, want_tiles: int = 0):
        """Fields per shared batch launch (1..16) and wave tiles per field
        (64..2^20); 0 restores a default."""
        _check(_load().pcrit_set_batch_config(self._ptr, int(group), int(want_tiles)),
               "set_batch_config")

    def batch_config(self):
        """(group, want_tiles) used by this context's batch calls."""
        g, w = ctypes.c_int(0), ctypes.c_int64(0)
        _check(_load().pcrit_get_batch_config(self._ptr, ctypes.byref(g), ctypes.byref(w)),
               "get_batch_config")
        return g.value, w.value

    def set_kernel_timing(self, levels=None):
        """Time the kernels of the given levels (iterable of ints), all
        levels (True), or none (None/False/empty)."""
        if levels is True:
            mask = (1 << 64) - 1
        elif not levels:
            mask = 0
        else:
            mask = 0
            for k in levels:
                mask |= 1 << int(k)
        _check(_load().pcrit_set_kernel_timing(self._ptr, mask),
               "set_kernel_timing")

    def kernel_ms(self, max_levels: int = 40):
        a = np.full(max_levels, -1, np.float32)
        b = np.full(max_levels, -1, np.float32)
        _check(_load().pcrit_kernel_ms(self._ptr, a.ctypes.data, b.ctypes.data,
                                       max_levels), "kernel_ms")
        return a, b


_default_ctx = {}


def _ctx_for(tensor, ctx):
    if ctx is not None:
        return ctx
    dev = tensor.device.index or 0
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def _stream_handle(tensor, stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(tensor.device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _check_field(field):
    import torch
    if not isinstance(field, torch.Tensor) or field.device.type != "cuda":
        raise PcritError(E_ARG, "field must be a torch tensor on a ROCm device")
    if field.dtype != torch.float32 or not field.is_contiguous():
        raise PcritError(E_ARG, "field must be contiguous float32")
    return _shape3(field.shape)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def check_buffer(name, t, dtype, device, *, numel=None, min_numel=None):
    """Reject a caller-supplied buffer that the library would write past or
    misread: wrong type, wrong device, not contiguous, or too small.  Raises
    PcritError(E_ARG) before anything is enqueued."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise PcritError(E_ARG, f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise PcritError(E_ARG, f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise PcritError(E_ARG, f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise PcritError(E_ARG, f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise PcritError(E_ARG, f"{name} must have {numel} elements, "
                                f"got {t.numel()}")
    if min_numel is not None and t.numel() < min_numel:
        raise PcritError(E_ARG, f"{name} must have at least {min_numel} "
                                f"elements, got {t.numel()}")
    return t


def _capacity(capacity, crit, default):
    """List capacity: as given, else the supplied list's length, else the
    default (enough for every vertex)."""
    if capacity is None:
        capacity = crit.numel() if crit is not None else default
    capacity = int(capacity)
    if capacity < 0:
        raise PcritError(E_ARG, "capacity must be >= 0")
    return capacity


@dataclass
class ClassifyResult:
    codes: "object"           # uint8 tensor, full resolution
    crit: "object"            # int32 tensor (uint32 values), ascending
    crit_codes: "object"      # uint8 tensor or None
    count: int                # number of critical vertices
    status: int


def classify(field, level: int = 0, *, ctx: Optional[Context] = None,
             capacity: Optional[int] = None, with_crit_codes: bool = False,
             codes=None, crit=None, stream=None, count_dev=None,
             check: bool = True) -> ClassifyResult:
    """Classify every vertex of level `level` of `field` (direct pass).

    With ``count_dev`` (an int64 device tensor of one element) the call is
    asynchronous and the count is written there; otherwise it synchronises
    and returns the count."""
    import torch
    nx, ny, nz = _check_field(field)
    lib = _load()
    c = _ctx_for(field, ctx)
    m = level_dims(field.shape, level)
    capacity = _capacity(capacity, crit, m[0] * m[1] * m[2])
    if codes is None:
        codes = torch.zeros(field.shape, dtype=torch.uint8, device=field.device)
    check_buffer("codes", codes, torch.uint8, field.device, numel=field.numel())
    if crit is None:
        crit = torch.empty(max(capacity, 1), dtype=torch.int32,
                           device=field.device)
    check_buffer("crit", crit, torch.int32, field.device, min_numel=capacity)
    if count_dev is not None:
        check_buffer("count_dev", count_dev, torch.int64, field.device,
                     min_numel=1)
    cc = (torch.empty(max(capacity, 1), dtype=torch.uint8, device=field.device)
          if with_crit_codes else None)
    cnt = ctypes.c_int64(-1)
    st = lib.pcrit_classify(
        c.handle, _stream_handle(field, stream), _ptr(field), nx, ny, nz,
        int(level), _ptr(codes), _ptr(crit), _ptr(cc), int(capacity),
        None if count_dev is not None else ctypes.byref(cnt), _ptr(count_dev))
    if check and st not in (0, E_CAPACITY):
        raise PcritError(st, "pcrit_classify")
    n = cnt.value
    if count_dev is not None:
        return ClassifyResult(codes, crit, cc, -1, st)
    k = max(0, min(n, capacity))
    return ClassifyResult(codes, crit[:k], None if cc is None else cc[:k], n,
                          st)


class _BatchField(ctypes.Structure):
    _fields_ = [("field", ctypes.c_void_p), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("codes", ctypes.c_void_p)]


@dataclass
class BatchResult:
    codes: List["object"]      # per field: uint8 tensor, full resolution
    crit: "object"             # int32 tensor: the lists of all fields
    crit_codes: "object"       # uint8 tensor or None
    offsets: np.ndarray        # n_fields + 1: field i's list is crit[off[i]:off[i+1]]
    status: int

    def field_list(self, i: int):
        return self.crit[int(self.offsets[i]):int(self.offsets[i + 1])]


def classify_batch(fields, *, ctx: Optional[Context] = None, capacity: Optional[int] = None,
                   with_crit_codes: bool = False, codes=None, crit=None, offsets_dev=None,
                   stream=None, check: bool = True) -> BatchResult:
    """Classify a list of fields (all 3D or all 2D, level 0) with shared
    launches.  With ``offsets_dev`` (int64 device tensor of n+1 elements)
    the call is asynchronous: offsets land there and ``offsets`` is None."""
    import torch
    if len(fields) < 1:
        raise PcritError(E_ARG, "empty batch")
    dev = fields[0].device
    lib = _load()
    c = _ctx_for(fields[0], ctx)
    descs = (_BatchField * len(fields))()
    total = 0
    out_codes = []
    for i, f in enumerate(fields):
        if f.device != dev:
            raise PcritError(E_ARG, "fields on different devices")
        nx, ny, nz = _check_field(f)
        cd = codes[i] if codes is not None else torch.zeros(f.shape, dtype=torch.uint8,
                                                             device=dev)
        check_buffer(f"codes[{i}]", cd, torch.uint8, dev, numel=f.numel())
        descs[i] = _BatchField(f.data_ptr(), nx, ny, nz, cd.data_ptr())
        out_codes.append(cd)
        total += f.numel()
    capacity = _capacity(capacity, crit, total)
    if crit is None:
        crit = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    check_buffer("crit", crit, torch.int32, dev, min_numel=capacity)
    cc = (torch.empty(max(capacity, 1), dtype=torch.uint8, device=dev)
          if with_crit_codes else None)
    if offsets_dev is not None:
        check_buffer("offsets_dev", offsets_dev, torch.int64, dev, min_numel=len(fields) + 1)
    offs = None if offsets_dev is not None else np.zeros(len(fields) + 1, np.int64)
    st = lib.pcrit_classify_batch(
        c.handle, _stream_handle(fields[0], stream), len(fields), ctypes.addressof(descs),
        _ptr(crit), _ptr(cc), int(capacity), None if offs is None else offs.ctypes.data,
        _ptr(offsets_dev))
    if check and st not in (0, E_CAPACITY):
        raise PcritError(st, "pcrit_classify_batch")
    return BatchResult(out_codes, crit, cc, offs, st)


BATCH_TUNE_GROUPS = (8, 16)
BATCH_TUNE_WANTS = (128, 256, 512, 1024, 2048, 4096)


def batch_autotune(fields, *, ctx: Optional[Context] = None, reps: int = 3,
                   capacity: Optional[int] = None, with_crit_codes: bool = False, stream=None):
    """pcrit_batch_autotune: time the batch call on these fields for every
    (group, want_tiles) in BATCH_TUNE_GROUPS x BATCH_TUNE_WANTS and keep the
    fastest in the context.  Returns ((group, want_tiles), {(group,
    want_tiles): ms per call}, codes, crit, crit_codes) -- the buffers hold
    the batch's result."""
    import torch
    if len(fields) < 1:
        raise PcritError(E_ARG, "empty batch")
    dev = fields[0].device
    c = _ctx_for(fields[0], ctx)
    descs = (_BatchField * len(fields))()
    total = 0
    out_codes = []
    for i, f in enumerate(fields):
        if f.device != dev:
            raise PcritError(E_ARG, "fields on different devices")
        nx, ny, nz = _check_field(f)
        cd = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
        descs[i] = _BatchField(f.data_ptr(), nx, ny, nz, cd.data_ptr())
        out_codes.append(cd)
        total += f.numel()
    capacity = _capacity(capacity, None, total)
    crit = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    cc = (torch.empty(max(capacity, 1), dtype=torch.uint8, device=dev)
          if with_crit_codes else None)
    times = np.zeros(len(BATCH_TUNE_GROUPS) * len(BATCH_TUNE_WANTS), np.float64)
    g, w = ctypes.c_int(0), ctypes.c_int64(0)
    _check(_load().pcrit_batch_autotune(
        c.handle, _stream_handle(fields[0], stream), len(fields), ctypes.addressof(descs),
        _ptr(crit), _ptr(cc), int(capacity), int(reps), times.ctypes.data, ctypes.byref(g),
        ctypes.byref(w)), "pcrit_batch_autotune")
    table = {(gi, wi): float(times[k]) for k, (gi, wi) in
             enumerate((gi, wi) for gi in BATCH_TUNE_GROUPS for wi in BATCH_TUNE_WANTS)}
    return (g.value, w.value), table, out_codes, crit, cc


def order_field(field, *, ctx: Optional[Context] = None, rank=None, sorted_out=None,
                stream=None):
    """(rank, sorted): the order field of ``field`` -- every vertex's rank by
    (value, index) -- and the vertex at each rank (int32 tensors holding
    uint32 values, flat)."""
    import torch
    nx, ny, nz = _check_field(field)
    c = _ctx_for(field, ctx)
    n = field.numel()
    if rank is None:
        rank = torch.empty(n, dtype=torch.int32, device=field.device)
    if sorted_out is None:
        sorted_out = torch.empty(n, dtype=torch.int32, device=field.device)
    check_buffer("rank", rank, torch.int32, field.device, numel=n)
    check_buffer("sorted_out", sorted_out, torch.int32, field.device, numel=n)
    _check(_load().pcrit_order_field(c.handle, _stream_handle(field, stream), _ptr(field), nx, ny,
                                     nz, _ptr(rank), _ptr(sorted_out)), "pcrit_order_field")
    return rank, sorted_out


def extrema(codes, *, ctx: Optional[Context] = None, capacity: Optional[int] = None,
            stream=None):
    """(minima, maxima) of full-resolution codes: ascending int32 tensors."""
    import torch
    if codes.dtype != torch.uint8 or not codes.is_contiguous():
        raise PcritError(E_ARG, "codes must be contiguous uint8")
    nx, ny, nz = _shape3(codes.shape)
    c = _ctx_for(codes, ctx)
    cap = codes.numel() * 2 if capacity is None else int(capacity)
    out = torch.empty(max(cap, 1), dtype=torch.int32, device=codes.device)
    cnt = np.zeros(2, np.int64)
    _check(_load().pcrit_extrema(c.handle, _stream_handle(codes, stream), _ptr(codes), nx, ny, nz,
                                 _ptr(out), cap, cnt.ctypes.data), "pcrit_extrema")
    a, b = int(cnt[0]), int(cnt[1])
    return out[:a], out[a:a + b]


LTS_SADDLE, LTS_PERSISTENT, LTS_BUDGET, LTS_INVALID = 0, 1, 2, 3
LTS_MAX_VISITED, LTS_MAX_FRONTIER = 32, 128


def lts_propagate(field, rank, extrema_list, *, maxima: bool = True,
                  epsilon: float = float("inf"), max_visited: int = 16, max_frontier: int = 64,
                  ctx: Optional[Context] = None, stream=None):
    """Step 1 of localized topological simplification: the superlevel
    (maxima) or sublevel (minima) set propagation from each listed extremum,
    with the persistence test.  ``rank`` is the order field (int32 tensor as
    order_field returns it), ``extrema_list`` int32 full-resolution indices.
    Returns (status uint8, saddle int32, visited int16) tensors, one entry
    per extremum; asynchronous on the stream."""
    import torch
    nx, ny, nz = _check_field(field)
    c = _ctx_for(field, ctx)
    check_buffer("rank", rank, torch.int32, field.device, numel=field.numel())
    check_buffer("extrema", extrema_list, torch.int32, field.device)
    n = extrema_list.numel()
    status = torch.empty(max(n, 1), dtype=torch.uint8, device=field.device)
    saddle = torch.empty(max(n, 1), dtype=torch.int32, device=field.device)
    visited = torch.empty(max(n, 1), dtype=torch.int16, device=field.device)
    _check(_load().pcrit_lts_propagate(
        c.handle, _stream_handle(field, stream), _ptr(field), _ptr(rank), nx, ny, nz,
        _ptr(extrema_list), n, 1 if maxima else 0, float(epsilon), int(max_visited),
        int(max_frontier), _ptr(status), _ptr(saddle), _ptr(visited)), "pcrit_lts_propagate")
    return status[:n], saddle[:n], visited[:n]


def lts_merged(field, rank, extrema_list, *, maxima: bool = True,
               epsilon: float = float("inf"), max_visited: int = 16, max_frontier: int = 64,
               ctx: Optional[Context] = None, stream=None):
    """Merged LTS Step 1 propagations (pcrit_lts_merged): propagations that
    meet at a saddle go on as one, led by the largest extremum; the others
    are paired with the saddle.  ``extrema_list`` holds distinct extrema of
    the kind asked for (as extrema() returns them).  Returns (status uint8,
    saddle int32, visited int16) tensors, one entry per listed extremum;
    asynchronous on the stream (the first call at a size grows the
    context's scratch)."""
    import torch
    nx, ny, nz = _check_field(field)
    c = _ctx_for(field, ctx)
    check_buffer("rank", rank, torch.int32, field.device, numel=field.numel())
    check_buffer("extrema", extrema_list, torch.int32, field.device)
    n = extrema_list.numel()
    status = torch.empty(max(n, 1), dtype=torch.uint8, device=field.device)
    saddle = torch.empty(max(n, 1), dtype=torch.int32, device=field.device)
    visited = torch.empty(max(n, 1), dtype=torch.int16, device=field.device)
    _check(_load().pcrit_lts_merged(
        c.handle, _stream_handle(field, stream), _ptr(field), _ptr(rank), nx, ny, nz,
        _ptr(extrema_list), n, 1 if maxima else 0, float(epsilon), int(max_visited),
        int(max_frontier), _ptr(status), _ptr(saddle), _ptr(visited)), "pcrit_lts_merged")
    return status[:n], saddle[:n], visited[:n]


def classify_noalloc(field, level: int, codes, crit, *, ctx: Context,
                     crit_codes=None, count_dev=None, stream=None,
                     check: bool = True) -> ClassifyResult:
    """pcrit_classify_noalloc: the direct pass with the library's fixed
    per-GPU scratch; the caller supplies every buffer (codes, crit, and
    optionally crit_codes and count_dev), so nothing is allocated here or in
    the library.  The capacity is the length of ``crit``.  Without
    ``count_dev`` the call synchronises and returns the count."""
    import torch
    nx, ny, nz = _check_field(field)
    lib = _load()
    check_buffer("codes", codes, torch.uint8, field.device, numel=field.numel())
    check_buffer("crit", crit, torch.int32, field.device)
    capacity = crit.numel()
    if crit_codes is not None:
        check_buffer("crit_codes", crit_codes, torch.uint8, field.device,
                     min_numel=capacity)
    if count_dev is not None:
        check_buffer("count_dev", count_dev, torch.int64, field.device,
                     min_numel=1)
    cnt = ctypes.c_int64(-1)
    st = lib.pcrit_classify_noalloc(
        ctx.handle, _stream_handle(field, stream), _ptr(field), nx, ny, nz,
        int(level), _ptr(codes), _ptr(crit), _ptr(crit_codes), int(capacity),
        None if count_dev is not None else ctypes.byref(cnt), _ptr(count_dev))
    if check and st not in (0, E_CAPACITY):
        raise PcritError(st, "pcrit_classify_noalloc")
    if count_dev is not None:
        return ClassifyResult(codes, crit, crit_codes, -1, st)
    n = cnt.value
    k = max(0, min(n, capacity))
    return ClassifyResult(codes, crit[:k],
                          None if crit_codes is None else crit_codes[:k], n, st)


@dataclass
class ProgressiveResult:
    codes: "object"
    crit: "object"              # concatenated lists, coarse to fine
    crit_codes: "object"
    levels: List[int]           # k_max .. 0
    offsets: np.ndarray         # k_max + 2 entries
    level_ms: Optional[np.ndarray]  # ms to each level's completion, or None
    reclassified: Optional[np.ndarray]  # old vertices re-classified per level
    status: int

    def level_list(self, level: int):
        i = self.levels.index(level)
        return self.crit[int(self.offsets[i]):int(self.offsets[i + 1])]

    def level_codes(self, level: int):
        i = self.levels.index(level)
        return self.crit_codes[int(self.offsets[i]):int(self.offsets[i + 1])]


def progressive(field, *, ctx: Optional[Context] = None,
                capacity: Optional[int] = None, with_crit_codes: bool = False,
                codes=None, crit=None, crit_codes=None, stream=None,
                callback=None, level_times: bool = False,
                count_reclassified: bool = False,
                check: bool = True) -> ProgressiveResult:
    """Coarse-to-fine classification over every level of the hierarchy.

    With ``level_times`` the result carries the stream time from the first
    kernel to each level's completion (level_ms); without, no events are
    recorded and level_ms is None.  With ``count_reclassified`` the result
    carries, per level, the number of old vertices whose polarity mask or
    absent set changed (``reclassified``; the library then tests every old
    vertex against the previous level); otherwise ``reclassified`` is
    None."""
    import torch
    nx, ny, nz = _check_field(field)
    lib = _load()
    c = _ctx_for(field, ctx)
    kmax, total = _hierarchy(tuple(field.shape))
    capacity = _capacity(capacity, crit, total)
    if codes is None:
        codes = torch.zeros(field.shape, dtype=torch.uint8, device=field.device)
    check_buffer("codes", codes, torch.uint8, field.device, numel=field.numel())
    if crit is None:
        crit = torch.empty(max(capacity, 1), dtype=torch.int32,
                           device=field.device)
    check_buffer("crit", crit, torch.int32, field.device, min_numel=capacity)
    if with_crit_codes and crit_codes is None:
        crit_codes = torch.empty(max(capacity, 1), dtype=torch.uint8,
                                 device=field.device)
    if crit_codes is not None:
        check_buffer("crit_codes", crit_codes, torch.uint8, field.device,
                     min_numel=capacity)
    offs = np.zeros(kmax + 2, np.int64)
    ms = np.zeros(kmax + 1, np.float32) if level_times else None
    rec = np.zeros(kmax + 1, np.int64) if count_reclassified else None
    cb = lib.LEVEL_CB(callback) if callback else lib.NULL_CB
    st = lib.pcrit_progressive(
        c.handle, _stream_handle(field, stream), _ptr(field), nx, ny, nz,
        _ptr(codes), _ptr(crit), _ptr(crit_codes), int(capacity),
        offs.ctypes.data, None if ms is None else ms.ctypes.data,
        None if rec is None else rec.ctypes.data, cb, None)
    if check and st not in (0, E_CAPACITY):
        raise PcritError(st, "pcrit_progressive")
    return ProgressiveResult(codes, crit, crit_codes,
                             list(range(kmax, -1, -1)), offs, ms, rec, st)


def progressive_async(field, *, ctx: Optional[Context] = None,
                      capacity: Optional[int] = None, codes=None, crit=None,
                      offsets=None, stream=None):
    """Enqueue a progressive classification without host synchronisation.

    Returns (codes, crit, offsets): offsets is a device int64 tensor of
    k_max+2 entries, valid once the stream reaches the end of the call's
    work (its last entry is -1 if the field had a NaN sample)."""
    import torch
    nx, ny, nz = _check_field(field)
    lib = _load()
    c = _ctx_for(field, ctx)
    kmax, total = _hierarchy(tuple(field.shape))
    capacity = _capacity(capacity, crit, total)
    if codes is None:
        codes = torch.zeros(field.shape, dtype=torch.uint8, device=field.device)
    check_buffer("codes", codes, torch.uint8, field.device, numel=field.numel())
    if crit is None:
        crit = torch.empty(max(capacity, 1), dtype=torch.int32, device=field.device)
    check_buffer("crit", crit, torch.int32, field.device, min_numel=capacity)
    if offsets is None:
        offsets = torch.empty(kmax + 2, dtype=torch.int64, device=field.device)
    check_buffer("offsets", offsets, torch.int64, field.device,
                 min_numel=kmax + 2)
    _check(lib.pcrit_progressive_async(
        c.handle, _stream_handle(field, stream), _ptr(field), nx, ny, nz,
        _ptr(codes), _ptr(crit), int(capacity), _ptr(offsets)),
        "pcrit_progressive_async")
    return codes, crit, offsets


def preview_f1(shape, level: int, preview, preview_codes, exact, exact_codes):
    """Host metric: (F1, matches) of a level-`level` preview list against the
    exact list (numpy uint32 indices, uint8 codes)."""
    nx, ny, nz = _shape3(shape)
    p = np.ascontiguousarray(preview, dtype=np.uint32)
    pc = np.ascontiguousarray(preview_codes, dtype=np.uint8)
    e = np.ascontiguousarray(exact, dtype=np.uint32)
    ec = np.ascontiguousarray(exact_codes, dtype=np.uint8)
    f1 = ctypes.c_double(0)
    mt = ctypes.c_int64(0)
    _check(_load().pcrit_preview_f1(nx, ny, nz, int(level), p.ctypes.data,
                                    pc.ctypes.data, len(p), e.ctypes.data,
                                    ec.ctypes.data, len(e), ctypes.byref(f1),
                                    ctypes.byref(mt)), "preview_f1")
    return f1.value, mt.value


def decode(codes):
    """(n_lower, n_upper, boundary, hole) arrays from code bytes."""
    c = np.asarray(codes).astype(np.int32)
    return c & 7, (c >> 3) & 7, (c >> 6) & 1, (c >> 7) & 1


def is_critical(codes):
    c = np.asarray(codes).astype(np.int32)
    return (c & 0xBF) != 0x09


def point_type(codes):
    """0 regular, 1 minimum, 2 maximum, 3 saddle."""
    nl, nu, _, hole = decode(codes)
    t = np.full(nl.shape, 3, np.int8)
    t[(nl == 1) & (nu == 1) & (hole == 0)] = 0
    t[nu == 0] = 2
    t[nl == 0] = 1
    return t


# ---------------------------------------------------------------------------
# Learned refinement order and region timeline
# ---------------------------------------------------------------------------
def region_count(shape, edge: int) -> int:
    nx, ny, nz = _shape3(shape)
    n = ctypes.c_int(0)
    _check(_load().pcrit_region_count(nx, ny, nz, int(edge), ctypes.byref(n)),
           "region_count")
    return n.value


def mlp_feature_level(shape) -> int:
    nx, ny, nz = _shape3(shape)
    k = ctypes.c_int(0)
    _check(_load().pcrit_mlp_feature_level(nx, ny, nz, ctypes.byref(k)),
           "mlp_feature_level")
    return k.value


def mlp_features(field, level: int, *, ctx: Optional[Context] = None, out=None,
                 stream=None):
    """Network inputs (n_level x 32, bfloat16) of every vertex of level
    ``level``."""
    import torch
    nx, ny, nz = _check_field(field)
    c = _ctx_for(field, ctx)
    m = level_dims(field.shape, level)
    n = m[0] * m[1] * m[2]
    if out is None:
        out = torch.empty((n, MLP_INPUTS), dtype=torch.bfloat16, device=field.device)
    check_buffer("out", out, torch.bfloat16, field.device, numel=n * MLP_INPUTS)
    _check(_load().pcrit_mlp_features(c.handle, _stream_handle(field, stream), _ptr(field),
                                      nx, ny, nz, int(level), _ptr(out)), "mlp_features")
    return out


def mlp_labels(codes, level: int, *, ctx: Optional[Context] = None, out=None,
               stream=None):
    """Training targets (uint8, ceil(255 x critical fraction of the cell)) of
    the vertices of level ``level`` from full-resolution level-0 codes."""
    import torch
    if codes.dtype != torch.uint8 or not codes.is_contiguous():
        raise PcritError(E_ARG, "codes must be contiguous uint8")
    nx, ny, nz = _shape3(codes.shape)
    c = _ctx_for(codes, ctx)
    m = level_dims(codes.shape, level)
    n = m[0] * m[1] * m[2]
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=codes.device)
    check_buffer("out", out, torch.uint8, codes.device, numel=n)
    _check(_load().pcrit_mlp_labels(c.handle, _stream_handle(codes, stream), _ptr(codes),
                                    nx, ny, nz, int(level), _ptr(out)), "mlp_labels")
    return out


def _check_params(params, device):
    import torch
    return check_buffer("params", params, torch.float32, device, numel=MLP_PARAMS)


def mlp_forward(params, X, *, ctx: Optional[Context] = None, out=None, stream=None):
    """Logits (float32) of the inputs X (n x 32 bfloat16)."""
    import torch
    check_buffer("X", X, torch.bfloat16, X.device)
    n = X.numel() // MLP_INPUTS
    _check_params(params, X.device)
    c = _ctx_for(X, ctx)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=X.device)
    check_buffer("out", out, torch.float32, X.device, min_numel=n)
    _check(_load().pcrit_mlp_forward(c.handle, _stream_handle(X, stream), _ptr(params),
                                     _ptr(X), n, _ptr(out)), "mlp_forward")
    return out


def mlp_backward(params, X, labels, *, ctx: Optional[Context] = None, grad=None,
                 loss=None, stream=None):
    """(grad, loss_sum): gradient of the mean binary cross-entropy."""
    import torch
    check_buffer("X", X, torch.bfloat16, X.device)
    n = X.numel() // MLP_INPUTS
    _check_params(params, X.device)
    check_buffer("labels", labels, torch.uint8, X.device, numel=n)
    c = _ctx_for(X, ctx)
    if grad is None:
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check_buffer("grad", grad, torch.float32, X.device, numel=MLP_PARAMS)
    check_buffer("loss", loss, torch.float32, X.device, min_numel=1)
    _check(_load().pcrit_mlp_backward(c.handle, _stream_handle(X, stream), _ptr(params),
                                      _ptr(X), _ptr(labels), n, _ptr(grad), _ptr(loss)),
           "mlp_backward")
    return grad, loss


def mlp_adam(params, grad, m, v, lr: float, step: int, *, ctx: Optional[Context] = None,
             stream=None):
    import torch
    for name, t in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        check_buffer(name, t, torch.float32, params.device, numel=MLP_PARAMS)
    c = _ctx_for(params, ctx)
    _check(_load().pcrit_mlp_adam(c.handle, _stream_handle(params, stream), _ptr(params),
                                  _ptr(grad), _ptr(m), _ptr(v), ctypes.c_float(lr),
                                  int(step)), "mlp_adam")


@dataclass
class TimelineResult:
    codes: "object"
    crit: "object"
    levels: List[int]
    offsets: np.ndarray
    level_ms: np.ndarray         # per level index i = k_max - k
    region_ms: np.ndarray        # (levels, regions)
    region_edge: int
    status: int
    rank: np.ndarray             # position of each region in the order used

    def level_list(self, level: int):
        i = self.levels.index(level)
        return self.crit[int(self.offsets[i]):int(self.offsets[i + 1])]


def progressive_timeline(field, region_edge: int = 64, *, order=None, params=None,
                         ctx: Optional[Context] = None, capacity: Optional[int] = None,
                         codes=None, crit=None, stream=None,
                         check: bool = True) -> TimelineResult:
    """Progressive classification with region-by-region refinement of the
    large levels and per-region completion times.  ``order``: None (region
    id order), or an int array of region ranks (rank[r] = position of
    region r); ``params``: the network's parameters (device float32) for the
    learned order (then ``order`` must be None)."""
    import torch
    nx, ny, nz = _check_field(field)
    lib = _load()
    c = _ctx_for(field, ctx)
    kmax, total = _hierarchy(tuple(field.shape))
    nreg = region_count(field.shape, region_edge)
    capacity = _capacity(capacity, crit, total)
    if codes is None:
        codes = torch.zeros(field.shape, dtype=torch.uint8, device=field.device)
    check_buffer("codes", codes, torch.uint8, field.device, numel=field.numel())
    if crit is None:
        crit = torch.empty(max(capacity, 1), dtype=torch.int32, device=field.device)
    check_buffer("crit", crit, torch.int32, field.device, min_numel=capacity)
    mode, rank = 0, None
    if params is not None:
        if order is not None:
            raise PcritError(E_ARG, "give either an order or network parameters")
        _check_params(params, field.device)
        mode = 2
        rank = np.zeros(nreg, np.int32)
    elif order is not None:
        rank = np.ascontiguousarray(order, dtype=np.int32)
        if rank.shape != (nreg,):
            raise PcritError(E_ARG, f"order must have {nreg} entries")
        mode = 1
    offs = np.zeros(kmax + 2, np.int64)
    lms = np.zeros(kmax + 1, np.float64)
    rms = np.zeros((kmax + 1, nreg), np.float64)
    st = lib.pcrit_progressive_timeline(
        c.handle, _stream_handle(field, stream), _ptr(field), nx, ny, nz, _ptr(codes),
        _ptr(crit), int(capacity), int(region_edge), mode,
        None if rank is None else rank.ctypes.data, _ptr(params), offs.ctypes.data,
        lms.ctypes.data, rms.ctypes.data)
    if check and st not in (0, E_CAPACITY):
        raise PcritError(st, "pcrit_progressive_timeline")
    return TimelineResult(codes, crit, list(range(kmax, -1, -1)), offs, lms, rms,
                          int(region_edge), st,
                          rank if rank is not None else np.arange(nreg, dtype=np.int32))


def preview_f1_levels(shape, preview, preview_codes, preview_levels, exact, exact_codes):
    """Host metric with a level per preview point: (F1, matches)."""
    nx, ny, nz = _shape3(shape)
    p = np.ascontiguousarray(preview, dtype=np.uint32)
    pc = np.ascontiguousarray(preview_codes, dtype=np.uint8)
    pl = np.ascontiguousarray(preview_levels, dtype=np.uint8)
    e = np.ascontiguousarray(exact, dtype=np.uint32)
    ec = np.ascontiguousarray(exact_codes, dtype=np.uint8)
    if not (len(p) == len(pc) == len(pl)) or len(e) != len(ec):
        raise PcritError(E_ARG, "list lengths differ")
    f1 = ctypes.c_double(0)
    mt = ctypes.c_int64(0)
    _check(_load().pcrit_preview_f1_levels(nx, ny, nz, p.ctypes.data, pc.ctypes.data,
                                           pl.ctypes.data, len(p), e.ctypes.data,
                                           ec.ctypes.data, len(e), ctypes.byref(f1),
                                           ctypes.byref(mt)), "preview_f1_levels")
    return f1.value, mt.value

