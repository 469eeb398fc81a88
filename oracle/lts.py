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

Merged propagations (``propagate_merged``), Sections 4.4 and 4.5: the
propagations meet at saddles.  A propagation that stops at a saddle s adds
to s's arrival count the higher neighbours of s it has taken; the one that
brings the count to the number of s's higher neighbours is the last to
arrive and carries on from s with the union of every arrived component, led
by the highest extremum among them; the leaders of the other arrived
components are paired with s (removed).  A propagation that no later
arrival takes over leaves its leader paired with the saddle where it
stopped.  Readings: the leader's value is the one the persistence test
uses; a merge that would hold `max_visited` vertices or more, or leave more
than `max_frontier` waiting, gives the leader BUDGET; a propagation whose
waiting set empties (the whole grid taken) makes its leader PERSISTENT (the
global extremum is never removed).  The result does not depend on which
propagation arrives last: the merged component and its waiting set are
unions, and the leader is the largest.

Pins (``tests/test_oracle_lts.py``): the component of a saddle stop equals
the connected component of the strict superlevel set of f-hat(s) containing
m, plus s, found by a breadth-first search (an independent definition); s
has a larger
neighbour outside it and is its smallest vertex; closed forms on fields
with one and with two bumps; the persistence rule against the value
difference of the saddle stop; minima are the maxima of -f.  Merged
propagations from every maximum with unbounded budgets remove exactly the
maxima whose elder-rule pair (a union-find sweep of the vertices in
decreasing order, written in the test) has a value difference of at most
epsilon, each at its paired saddle; processing the propagations in any
order gives the same result.
"""
from __future__ import annotations

import numpy as np

from .order import order_field

# Freudenthal neighbours (dx, dy, dz): the seven "positive" offsets and
# their negatives; in 2D the three positive offsets of the (1, 1) diagonal
_POS3 = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]
_POS2 = [(1, 0, 0), (0, 1, 0), (1, 1, 0)]

SADDLE, PERSISTENT, BUDGET, INVALID = 0, 1, 2, 3


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


def propagate_merged(f, extrema, eps, maxima=True, max_visited=16, max_frontier=64, rank=None,
                     order=None):
    """Merged propagations from every listed extremum (Sections 4.4, 4.5):
    (status uint8, saddle int32, visited uint16) per listed extremum.
    The listed vertices must be distinct.  status: SADDLE with the saddle
    the extremum is paired with (removed), PERSISTENT, BUDGET, or INVALID
    for an index outside the grid or a vertex that is not an extremum of
    the kind asked for (some neighbour comes later in the order); visited:
    the vertices of the component the extremum led when its status was set.
    `order`: the order in which the propagations start (any order gives the
    same result; the pins use it)."""
    f = np.asarray(f, dtype=np.float32)
    shape = f.shape
    fv = f.ravel()
    if rank is None:
        rank, _ = order_field(f)
    key = rank.astype(np.int64) if maxima else (rank.size - 1 - rank.astype(np.int64))
    ext = np.asarray(extrema, dtype=np.int64)
    n = len(ext)
    status = np.full(n, INVALID, np.uint8)
    saddle = np.full(n, -1, np.int32)
    visited = np.zeros(n, np.uint16)
    diff = (lambda top, v: np.float32(fv[top] - fv[v])) if maxima else \
        (lambda top, v: np.float32(fv[v] - fv[top]))

    # one propagation: leader (index into ext), component, waiting vertices
    work = []
    for i in (range(n) if order is None else order):
        m = int(ext[i])
        if 0 <= m < fv.size and all(key[u] < key[m] for u in neighbours(shape, m)):
            work.append((i, {m}, {u: int(key[u]) for u in neighbours(shape, m)}))
    arrivals = {}  # saddle -> [count of its higher neighbours taken, parked propagations]

    def finish(lead, st, s, size):
        status[lead], saddle[lead], visited[lead] = st, s, size

    while work:
        lead, comp, front = work.pop()
        while True:
            if not front:
                finish(lead, PERSISTENT, -1, len(comp))
                break
            v = max(front, key=front.get)
            del front[v]
            comp.add(v)
            if diff(int(ext[lead]), v) > np.float32(eps):
                finish(lead, PERSISTENT, -1, len(comp))
                break
            higher = [u for u in neighbours(shape, v) if key[u] > key[v]]
            mine = sum(1 for u in higher if u in comp)
            if mine < len(higher):  # v is a saddle: arrive there
                finish(lead, SADDLE, v, len(comp))
                arr = arrivals.setdefault(v, [0, []])
                arr[0] += mine
                arr[1].append((lead, comp, front))
                if arr[0] < len(higher):
                    break
                # the last arrival: merge every arrived propagation at v
                parts = arr[1]
                del arrivals[v]
                lead = max((p[0] for p in parts), key=lambda j: key[int(ext[j])])
                comp = set().union(*(p[1] for p in parts))
                front = {}
                for p in parts:
                    front.update(p[2])
                front.update({u: int(key[u]) for u in neighbours(shape, v)})
                front = {u: k for u, k in front.items() if u not in comp}
                if len(comp) >= max_visited or len(front) > max_frontier:
                    finish(lead, BUDGET, -1, len(comp))
                    break
                continue
            if len(comp) >= max_visited:
                finish(lead, BUDGET, -1, len(comp))
                break
            for u in neighbours(shape, v):
                if u not in comp and u not in front:
                    front[u] = int(key[u])
            if len(front) > max_frontier:
                finish(lead, BUDGET, -1, len(comp))
                break
    return status, saddle, visited
