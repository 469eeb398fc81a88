"""CPU oracle for PL critical-point classification (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code or table with it.

The arithmetic lives in ``pcrit_oracle.c`` (plain C, explicit link per
vertex, union-find component counts); this module builds it with gcc and wraps
it with ctypes.  It follows Section 3.1 (star, link, lower/upper link,
regular/critical, saddles) and Section 4.1 (ties broken by memory position) of
Lukasczyk et al., "Localized Topological Simplification of Scalar Data".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcrit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_DIMS, E_LEVEL, E_CAPACITY, E_NAN, E_OOM = 0, -1, -2, -3, -4, -5, -7

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    global _lib
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-pthread", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32 = ctypes.c_int64, ctypes.c_int
    vp = ctypes.c_void_p
    lib.oracle_classify.argtypes = [vp, i64, i64, i64, i32, i64, i64, vp, vp,
                                    vp, vp, i64, ctypes.POINTER(i64), i32]
    lib.oracle_classify.restype = i32
    lib.oracle_vertex_detail.argtypes = [vp, i64, i64, i64, i32, i64, vp, vp]
    lib.oracle_vertex_detail.restype = i32
    lib.oracle_level_dims.argtypes = [i64, i64, i64, i32, vp]
    lib.oracle_level_dims.restype = i32
    lib.oracle_classify_link.argtypes = [i32, vp, i32, vp, i32, vp, i32, i32,
                                         vp]
    lib.oracle_classify_link.restype = i32
    _lib = lib
    return lib


def _dims(field):
    if field.ndim == 3:
        nz, ny, nx = field.shape
    elif field.ndim == 2:
        (ny, nx), nz = field.shape, 1
    else:
        raise ValueError("field must be 2D (ny, nx) or 3D (nz, ny, nx)")
    return int(nx), int(ny), int(nz)


def level_dims(shape, level):
    """Samples per axis (x, y, z) of level `level` for a C-order shape."""
    lib = _load()
    if len(shape) == 3:
        nz, ny, nx = shape
    else:
        (ny, nx), nz = shape, 1
    m = np.zeros(3, np.int64)
    st = lib.oracle_level_dims(nx, ny, nz, level, m.ctypes.data)
    if st:
        raise ValueError(f"invalid level {level} for shape {shape} ({st})")
    return tuple(int(v) for v in m)


def max_level(shape):
    dims = [d for d in shape if d > 1] if len(shape) == 3 else list(shape)
    k = 0
    while all((1 << (k + 1)) <= d - 1 for d in dims):
        k += 1
    return k


class Result:
    """codes: full-resolution uint8 array (only level positions meaningful);
    crit: ascending uint32 full-resolution indices of critical vertices;
    status: 0 or a negative error code."""

    def __init__(self, codes, crit, status, chi_lower=None, chi_upper=None):
        self.codes = codes
        self.crit = crit
        self.status = status
        self.chi_lower = chi_lower
        self.chi_upper = chi_upper


def classify(field, level=0, slow_range=None, want_chi=False, threads=None,
             codes=None, cap=None):
    """Classify every vertex of level `level` (stride 2^level).

    ``slow_range = (b, e)`` restricts to level-local z (3D) or y (2D) in
    [b, e) -- the bench uses it to time a bounded sample.
    """
    lib = _load()
    f = np.ascontiguousarray(field, dtype=np.float32)
    nx, ny, nz = _dims(f)
    m = level_dims(f.shape, level)
    nloc = m[0] * m[1] * m[2]
    if codes is None:
        codes = np.zeros(f.shape, np.uint8)
    b, e = slow_range if slow_range is not None else (0, -1)
    if cap is None:
        cap = nloc
    crit = np.zeros(max(cap, 1), np.uint32)
    chil = np.zeros(nloc, np.int8) if want_chi else None
    chiu = np.zeros(nloc, np.int8) if want_chi else None
    cnt = ctypes.c_int64(0)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    st = lib.oracle_classify(
        f.ctypes.data, nx, ny, nz, level, b, e, codes.ctypes.data,
        chil.ctypes.data if want_chi else None,
        chiu.ctypes.data if want_chi else None,
        crit.ctypes.data, cap, ctypes.byref(cnt), threads)
    if st not in (OK, E_CAPACITY, E_NAN):
        raise ValueError(f"oracle_classify failed with status {st}")
    n = min(cnt.value, cap)
    res = Result(codes, crit[:n].copy(), st, chil, chiu)
    res.count = cnt.value
    return res


DETAIL_FIELDS = ("code", "n_lower", "n_upper", "chi_lower", "chi_upper",
                 "b1_lower", "b1_upper", "boundary", "nsc", "critical",
                 "link_v", "link_ef")


def vertex_detail(field, coords, level=0):
    """Per-vertex link statistics; coords are level-local (x, y, z) rows.
    Returns an int array of shape (len(coords), 12), columns DETAIL_FIELDS
    (link_ef = #edges + 1000 * #triangles)."""
    lib = _load()
    f = np.ascontiguousarray(field, dtype=np.float32)
    nx, ny, nz = _dims(f)
    c = np.ascontiguousarray(np.asarray(coords, dtype=np.int64).reshape(-1, 3))
    out = np.zeros((c.shape[0], 12), np.int32)
    st = lib.oracle_vertex_detail(f.ctypes.data, nx, ny, nz, level,
                                  c.shape[0], c.ctypes.data, out.ctypes.data)
    if st:
        raise ValueError(f"oracle_vertex_detail failed with status {st}")
    return out


def classify_link(lower, edges, tris=(), link_dim=1, closed=True):
    """Classify a vertex from an explicit link complex.

    lower[i] is True if link vertex i comes before the vertex in the order.
    Returns (critical, dict of n_lower, n_upper, chi_lower, chi_upper,
    b1_lower, b1_upper)."""
    lib = _load()
    lo = np.ascontiguousarray(np.asarray(lower, dtype=np.int32))
    ed = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    tr = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(6, np.int32)
    st = lib.oracle_classify_link(lo.shape[0], lo.ctypes.data, ed.shape[0],
                                  ed.ctypes.data, tr.shape[0], tr.ctypes.data,
                                  link_dim, int(bool(closed)), out.ctypes.data)
    if st < 0:
        raise ValueError(f"oracle_classify_link failed with status {st}")
    keys = ("n_lower", "n_upper", "chi_lower", "chi_upper", "b1_lower",
            "b1_upper")
    return bool(st), dict(zip(keys, (int(v) for v in out)))


def decode(codes):
    """Split code bytes into (n_lower, n_upper, boundary, nsc) arrays."""
    c = np.asarray(codes).astype(np.int32)
    return c & 7, (c >> 3) & 7, (c >> 6) & 1, (c >> 7) & 1


def is_critical_code(codes):
    nl, nu, _, nsc = decode(codes)
    return ~((nl == 1) & (nu == 1) & (nsc == 0))
