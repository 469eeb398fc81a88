"""CPU oracle of Step 1 of localized topological simplification: the
superlevel (sublevel) set propagation from an extremum (test
infrastructure: only the tests and bench.py's CPU baseline use it; the GPU
library never imports it).

Section 4.2, Step 1: the component of the superlevel set of the order field
that a maximum m starts is grown one vertex at a time, always taking the
largest vertex adjacent to the component, until the vertex just taken has a
larger neighbour outside the component: that vertex is the saddle s where
m's component meets another one, and the component is the vertex set of the
strict superlevel set of f-hat(s) that contains m, together with s.  Minima: the same with the order
reversed (sublevel sets).  Section 4.5 adds a persistence test: the
propagation follows the value difference between m and the vertex it just
took, and stops as soon as that exceeds epsilon (m is then persistent).

Readings (the paper is silent on them): the order is the order field
(value, then memory index); the difference is taken in float32 on the
original values; it is tested before the saddle test, so a saddle reached
with a difference above epsilon makes m persistent; each extremum
propagates on its own (the merging of propagations at shared saddles is not
part of this step); the propagation gives up ("budget") once the component
holds `max_visited` vertices or more than `max_frontier` vertices wait
outside it.

Pins (``tests/test_oracle_lts.py``): the component of a saddle stop equals
the connected component of the strict superlevel set of f-hat(s) containing
m, plus s, found by a breadth-first search (an independent definition); s
has a larger
neighbour outside it and is its smallest vertex; closed forms on fields
with one and with two bumps; the persistence rule against the value
difference of the saddle stop; minima are the maxima of -f.
"""
from __future__ import annotations

import numpy as np

from .order import order_field

# Freudenthal neighbours (dx, dy, dz): the seven "positive" offsets and
# their negatives; in 2D the three positive offsets of the (1, 1) diagonal
_POS3 = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
_POS2 = [(1, 0, 0), (0, 1, 0), (1, 1, 0)]

SADDLE, PERSISTENT, BUDGET = 0, 1, 2


def _offsets(dim):
    pos = _POS3 if dim == 3 else _POS2
    return pos + [tuple(-c for c in p) for p in pos]


def _grid(shape):
    """(nx, ny, nz, dim) of a C-order array shaped (nz, ny, nx) or (ny, nx)."""
    if len(shape) == 3:
        return shape[2], shape[1], shape[0], 3
    return shape[1], shape[0], 1, 2


def neighbours(shape, v):
    nx, ny, nz, dim = _grid(shape)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    out = []
    for dx, dy, dz in _offsets(dim):
        a, b, c = x + dx, y + dy, z + dz
        if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
            out.append(int((c * ny + b) * nx + a))
    return out


def propagate(f, key, shape, m, eps, max_visited=16, max_frontier=64, maxima=True):
    """Propagation from extremum m.  key: the order (rank) to grow along,
    larger first (for minima pass the reversed rank).  Returns
    (status, saddle or -1, visited count)."""
    st, s, comp = propagate_set(f, key, shape, m, eps, max_visited, max_frontier, maxima)
    return st, s, len(comp)


def propagate_all(f, extrema, eps, maxima=True, max_visited=16, max_frontier=64, rank=None):
    """Propagations from every listed extremum: (status uint8, saddle int32,
    visited uint16) arrays."""
    f = np.asarray(f, dtype=np.float32)
    if rank is None:
        rank, _ = order_field(f)
    key = rank.astype(np.int64) if maxima else (rank.size - 1 - rank.astype(np.int64))
    n = len(extrema)
    st = np.zeros(n, np.uint8)
    sd = np.full(n, -1, np.int32)
    vi = np.zeros(n, np.uint16)
    for i, m in enumerate(np.asarray(extrema, dtype=np.int64)):
        a, b, c = propagate(f, key, f.shape, int(m), eps, max_visited, max_frontier, maxima)
        st[i], sd[i], vi[i] = a, b, c
    return st, sd, vi


def superlevel_component(shape, key, m, level):
    """Vertices of the connected component of {u: key(u) >= level} that
    contains m (a search over the Freudenthal neighbours; for the pins)."""
    seen = {m}
    todo = [m]
    while todo:
        v = todo.pop()
        for u in neighbours(shape, v):
            if u not in seen and key[u] >= level:
                seen.add(u)
                todo.append(u)
    return seen


def propagate_set(f, key, shape, m, eps, max_visited=16, max_frontier=64, maxima=True):
    """(status, saddle or -1, the set of vertices taken): start with m and
    its neighbours waiting; take the largest waiting vertex v; stop if
    f(m) - f(v) > eps (persistent), if v has a larger neighbour not taken
    (saddle v), or at the budget; else let v's neighbours wait too."""
    fv = np.asarray(f, dtype=np.float32).ravel()
    fm = fv[m]
    cs = {m}
    front = {u: int(key[u]) for u in neighbours(shape, m)}
    while front:
        v = max(front, key=front.get)
        del front[v]
        cs.add(v)
        d = np.float32(fm - fv[v]) if maxima else np.float32(fv[v] - fm)
        if d > np.float32(eps):
            return PERSISTENT, -1, cs
        nb = neighbours(shape, v)
        if any(u not in cs and key[u] > key[v] for u in nb):
            return SADDLE, v, cs
        if len(cs) >= max_visited:
            return BUDGET, -1, cs
        for u in nb:
            if u not in cs and u not in front:
                front[u] = int(key[u])
        if len(front) > max_frontier:
            return BUDGET, -1, cs
    return BUDGET, -1, cs
