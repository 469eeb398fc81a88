"""Brute-force reference on tiny grids, independent of the oracle's code.

The triangulation is described here in a different way from the oracle's
cell-by-cell tetrahedra: a set of grid points is a simplex iff it is a chain
p0 < p1 < ... < pk in the componentwise order with pk - p0 in {0,1}^d (the
Kuhn/Freudenthal description).  Everything is enumerated globally, so the link
of v is simply {sigma minus v : v in sigma}.  Only for grids of a few dozen
points.
"""
from __future__ import annotations

import itertools

import numpy as np


def grid_points(shape_xyz):
    return list(itertools.product(*[range(n) for n in shape_xyz]))


def simplices(shape_xyz):
    """All simplices (tuples of points, sorted along the chain)."""
    d = len(shape_xyz)
    steps = [s for s in itertools.product((0, 1), repeat=d) if any(s)]
    pts = set(grid_points(shape_xyz))
    out = []

    def grow(chain):
        out.append(tuple(chain))
        p0 = chain[0]
        last = chain[-1]
        for s in steps:
            q = tuple(a + b for a, b in zip(last, s))
            if q not in pts:
                continue
            if all(0 <= qa - pa <= 1 for qa, pa in zip(q, p0)):
                grow(chain + [q])

    for p in sorted(pts):
        grow([p])
    return out


def order_key(field_xyz, shape_xyz):
    """key(p) = (f(p), linear index with x fastest)."""
    def key(p):
        idx = 0
        mul = 1
        for a, n in zip(p, shape_xyz):
            idx += a * mul
            mul *= n
        return (float(field_xyz[p]), idx)
    return key


def components(vertices, edges):
    parent = {v: v for v in vertices}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return len({find(v) for v in vertices})


class Complex:
    def __init__(self, shape_xyz):
        self.shape = tuple(shape_xyz)
        self.simp = simplices(self.shape)
        self.star = {}
        for s in self.simp:
            for p in s:
                self.star.setdefault(p, []).append(s)

    def link(self, v):
        out = []
        for s in self.star[v]:
            if len(s) > 1:
                out.append(tuple(p for p in s if p != v))
        return out

    def vertex_stats(self, field_xyz, v):
        """(n_lower, n_upper, chi_lower, chi_upper, delta_chi) for vertex v.

        delta_chi = sum over simplices whose highest vertex is v of
        (-1)^dim: the change of the Euler characteristic of the sublevel
        complex when v is added."""
        key = order_key(field_xyz, self.shape)
        kv = key(v)
        lk = self.link(v)
        res = []
        for lower in (True, False):
            part = [s for s in lk
                    if all((key(p) < kv) == lower for p in s)]
            verts = [s[0] for s in part if len(s) == 1]
            edges = [s for s in part if len(s) == 2]
            chi = sum((-1) ** (len(s) - 1) for s in part)
            res.append((components(verts, edges), chi))
        dchi = 0
        for s in self.star[v]:
            if max(key(p) for p in s) == kv:
                dchi += (-1) ** (len(s) - 1)
        return res[0][0], res[1][0], res[0][1], res[1][1], dchi


def field_xyz(field_czyx):
    """C-order (z,y,x) or (y,x) numpy array -> dict keyed by (x,y[,z])."""
    a = np.asarray(field_czyx)
    if a.ndim == 3:
        nz, ny, nx = a.shape
        return {(x, y, z): a[z, y, x] for z in range(nz) for y in range(ny)
                for x in range(nx)}, (nx, ny, nz)
    ny, nx = a.shape
    return {(x, y): a[y, x] for y in range(ny) for x in range(nx)}, (nx, ny)


def gf2_rank(rows):
    """Rank over GF(2) of a matrix given as a list of int bit-rows."""
    rank = 0
    rows = [r for r in rows if r]
    while rows:
        pivot = rows.pop()
        if not pivot:
            continue
        rank += 1
        low = pivot & -pivot
        rows = [r ^ pivot if r & low else r for r in rows]
        rows = [r for r in rows if r]
    return rank


def betti(complex_simplices):
    """(b0, b1, b2) over GF(2) of a simplicial complex given as a set of
    simplices (tuples of hashable vertices, closed under faces)."""
    by_dim = {}
    for s in complex_simplices:
        by_dim.setdefault(len(s) - 1, []).append(tuple(sorted(s)))
    idx = {d: {s: i for i, s in enumerate(v)} for d, v in by_dim.items()}

    def boundary_rank(d):
        if d not in by_dim or (d - 1) not in by_dim:
            return 0
        rows = []
        for s in by_dim[d]:
            r = 0
            for i in range(len(s)):
                face = s[:i] + s[i + 1:]
                r |= 1 << idx[d - 1][face]
            rows.append(r)
        return gf2_rank(rows)

    n = [len(by_dim.get(d, [])) for d in range(3)]
    r1, r2, r3 = boundary_rank(1), boundary_rank(2), boundary_rank(3)
    return (n[0] - r1, n[1] - r1 - r2, n[2] - r2 - r3)


def link_part_betti(cplx, field_xyz, v, lower):
    key = order_key(field_xyz, cplx.shape)
    kv = key(v)
    part = [s for s in cplx.link(v)
            if all((key(p) < kv) == lower for p in s)]
    return betti(part)
