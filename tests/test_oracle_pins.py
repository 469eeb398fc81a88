"""Pins of the CPU oracle against facts fixed by the paper and by topology.

None of these expected values comes from the oracle itself or from the GPU
path: they are the paper's Fig. 3, theorems (Euler characteristic of the
sublevel filtration, Alexander duality on the 2-sphere), closed forms for
linear and separable fields, exact probabilities for i.i.d. fields, and an
independent brute force on tiny grids (``tests/bruteforce.py``).
"""
import itertools
import json
import os

import numpy as np
import pytest

import fieldgen
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# The 14 neighbour offsets (dx, dy, dz) of the grid triangulation and the 6 of
# the 2D one: differences in +-({0,1}^d \ 0).  Test-side only.
N14 = [d for d in itertools.product((-1, 0, 1), repeat=3)
       if any(d) and (all(c >= 0 for c in d) or all(c <= 0 for c in d))]
N6 = [d for d in itertools.product((-1, 0, 1), repeat=2)
      if any(d) and (all(c >= 0 for c in d) or all(c <= 0 for c in d))]


# --------------------------------------------------------------------------
# Fig. 3: the paper's drawn examples
# --------------------------------------------------------------------------
def test_fig_cp_golden(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "fig_cp.json")))
    # the link is the set of faces of star triangles that do not contain v
    names = sorted({p for t in g["star_triangles"] for p in t if p != "v"})
    ids = {n: i for i, n in enumerate(names)}
    edges = sorted({tuple(sorted(ids[p] for p in t if p != "v"))
                    for t in g["star_triangles"]})
    assert len(edges) == 5  # a closed 5-cycle around v
    for case in g["cases"]:
        lower = [case["signs"][n] == "-" for n in names]
        crit, r = oracle_mod.classify_link(lower, edges, link_dim=1,
                                           closed=True)
        assert r["n_lower"] == case["n_lower"], case["panel"]
        assert r["n_upper"] == case["n_upper"], case["panel"]
        kind = ("regular" if not crit else "minimum" if r["n_lower"] == 0
                else "maximum" if r["n_upper"] == 0 else "saddle")
        assert kind == case["type"], case["panel"]


# --------------------------------------------------------------------------
# Link shapes: a 2-sphere inside, a disk on the boundary
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(3, 3, 3), (2, 3, 4), (2, 2, 2), (4, 2, 3)])
def test_link_is_sphere_or_disk_3d(oracle_mod, shape):
    nz, ny, nx = shape
    f = np.zeros(shape, np.float32)
    coords = [(x, y, z) for z in range(nz) for y in range(ny)
              for x in range(nx)]
    d = oracle_mod.vertex_detail(f, coords)
    for (x, y, z), row in zip(coords, d):
        V, E, F = row[10], row[11] % 1000, row[11] // 1000
        interior = 0 < x < nx - 1 and 0 < y < ny - 1 and 0 < z < nz - 1
        assert row[7] == (not interior)
        if interior:
            # 14 neighbours, closed surface (3F = 2E), chi(S^2) = 2
            assert (V, E, F) == (14, 36, 24)
        else:
            assert V - E + F == 1  # a disk
            assert 3 * F < 2 * E


def test_link_is_circle_or_path_2d(oracle_mod):
    f = np.zeros((4, 5), np.float32)
    coords = [(x, y, 0) for y in range(4) for x in range(5)]
    d = oracle_mod.vertex_detail(f, coords)
    for (x, y, _), row in zip(coords, d):
        V, E = row[10], row[11] % 1000
        interior = 0 < x < 4 and 0 < y < 3
        if interior:
            assert (V, E) == (6, 6)
        else:
            assert V - E == 1  # a path


# --------------------------------------------------------------------------
# Every interior polarity pattern (2^14 of them)
# --------------------------------------------------------------------------
def packed_interior_patterns():
    """A grid of 16384 disjoint 3x3x3 blocks; block b's centre has value 0 and
    its neighbour N14[j] value +1 if bit j of b is set (upper), -1 otherwise.
    Returns (field (z,y,x), centre coordinates (x,y,z) per pattern)."""
    bx, by, bz = 32, 32, 16
    f = np.full((3 * bz, 3 * by, 3 * bx), 0.5, np.float32)
    centres = []
    for b in range(1 << 14):
        cx, cy, cz = 3 * (b % bx) + 1, 3 * ((b // bx) % by) + 1, 3 * (b // (bx * by)) + 1
        f[cz, cy, cx] = 0.0
        for j, (dx, dy, dz) in enumerate(N14):
            f[cz + dz, cy + dy, cx + dx] = 1.0 if (b >> j) & 1 else -1.0
        centres.append((cx, cy, cz))
    return f, np.array(centres)


@pytest.fixture(scope="module")
def interior_patterns(oracle_mod):
    f, centres = packed_interior_patterns()
    d = oracle_mod.vertex_detail(f, centres)
    return f, centres, d


def test_exhaustive_interior_duality(interior_patterns):
    _, _, d = interior_patterns
    nl, nu, chil, chiu = d[:, 1], d[:, 2], d[:, 3], d[:, 4]
    masks = np.arange(1 << 14)
    # exactly one minimum (all upper) and one maximum (all lower)
    assert np.flatnonzero(nl == 0).tolist() == [(1 << 14) - 1]
    assert np.flatnonzero(nu == 0).tolist() == [0]
    # Alexander duality on the link 2-sphere: b1(Lk-) = #components(Lk+) - 1,
    # hence chi(Lk-) = #L - (#U - 1) whenever both parts are non-empty
    mid = (nl > 0) & (nu > 0)
    assert np.array_equal(chil[mid], nl[mid] - nu[mid] + 1)
    assert np.array_equal(chiu[mid], nu[mid] - nl[mid] + 1)
    assert chil[nl == 0].tolist() == [0] and chil[nu == 0].tolist() == [2]
    b1l, b1u = d[:, 5], d[:, 6]
    assert np.array_equal(b1l[mid], nu[mid] - 1)
    assert np.array_equal(b1u[mid], nl[mid] - 1)
    # the whole link (a 2-sphere) and the empty set have no 1-cycles
    assert b1l[nu == 0].tolist() == [0] and b1u[nl == 0].tolist() == [0]
    # swapping upper and lower (complementing the mask) swaps #L and #U
    comp = ((1 << 14) - 1) ^ masks
    assert np.array_equal(nl, nu[comp])
    # interior vertices never get the non-simply-connected flag, and the code
    # is #L | #U << 3
    assert np.array_equal(d[:, 0], nl | (nu << 3))


def test_exhaustive_interior_matches_bruteforce(interior_patterns):
    """Component counts of every pattern against the chain-based brute force
    on one 3x3x3 grid."""
    cplx = bf.Complex((3, 3, 3))
    centre = (1, 1, 1)
    lk = cplx.link(centre)
    lverts = [s[0] for s in lk if len(s) == 1]
    ledges = [s for s in lk if len(s) == 2]
    assert len(lverts) == 14 and len(ledges) == 36
    pos = {(1 + dx, 1 + dy, 1 + dz): j for j, (dx, dy, dz) in enumerate(N14)}
    _, _, d = interior_patterns
    for b in range(1 << 14):
        up = {p for p in lverts if (b >> pos[p]) & 1}
        lo = [p for p in lverts if p not in up]
        nl = bf.components(lo, [e for e in ledges if e[0] not in up and e[1] not in up])
        nu = bf.components(list(up), [e for e in ledges if e[0] in up and e[1] in up])
        assert (d[b, 1], d[b, 2]) == (nl, nu), b


# --------------------------------------------------------------------------
# Euler characteristic of the sublevel filtration
# --------------------------------------------------------------------------
EULER_SHAPES = [(5, 4, 3), (2, 2, 2), (3, 7, 2), (6, 5, 4), (9, 8), (2, 2),
                (3, 11), (17, 5)]


@pytest.mark.parametrize("shape", EULER_SHAPES)
@pytest.mark.parametrize("levels", [2, 3, 1000])
def test_euler_sum_is_one(oracle_mod, shape, levels):
    """Adding v to the sublevel complex changes chi by 1 - chi(Lk-(v)); after
    all vertices the complex is the (contractible) box, so the sum is 1.  The
    same holds for the superlevel filtration with Lk+.  Heavy ties test the
    index tie-break."""
    for seed in range(3):
        f = fieldgen.tie_field(shape, seed, levels)
        r = oracle_mod.classify(f, want_chi=True, threads=2)
        assert np.sum(1 - r.chi_lower.astype(np.int64)) == 1
        assert np.sum(1 - r.chi_upper.astype(np.int64)) == 1


def _morse_count(codes, dim):
    nl, nu, _, _ = (np.asarray(x, np.int64) for x in
                    (codes & 7, (codes >> 3) & 7, 0, 0))
    mins = (nl == 0).sum()
    maxs = (nu == 0).sum()
    m1 = np.maximum(nl - 1, 0).sum()
    m2 = np.maximum(nu - 1, 0).sum()
    if dim == 3:
        return int(mins - m1 + m2 - maxs)
    return int(mins + maxs - m1)


@pytest.mark.parametrize("shape", [(9, 10, 11), (6, 13, 7), (31, 29), (40, 3)])
@pytest.mark.parametrize("pad", [np.inf, -np.inf])
def test_padded_morse_count(oracle_mod, shape, pad):
    """Pad by one layer of +inf (or -inf) so every original vertex is
    interior.  With +inf padding the original vertices come first and fill a
    closed box (chi = 1); with -inf they come after a shell with chi = chi of
    a sphere (2 in 3D, 0 in 2D).  So over the original vertices
    #min - sum m1 + sum m2 - #max = 1 (+inf) / -1 (-inf) in 3D, and
    #min + #max - sum m = 1 in 2D, saddles counted with multiplicity."""
    dim = len(shape)
    for seed, gen in [(0, "tie"), (1, "iid"), (2, "gauss")]:
        if gen == "tie":
            f = fieldgen.tie_field(shape, seed, 3)
        elif gen == "iid":
            f = fieldgen.iid_field(shape, seed)
        else:
            f = fieldgen.gaussian_field(shape, seed, 6, noise=("uniform", 1e-3))
        p = np.pad(f, 1, constant_values=pad).astype(np.float32)
        r = oracle_mod.classify(p)
        inner = r.codes[(slice(1, -1),) * dim]
        expect = (1 if pad > 0 else -1) if dim == 3 else 1
        assert _morse_count(inner, dim) == expect


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
def _argext(f, level=0):
    """Full-resolution indices of the first and last level vertex in the
    order (value, index)."""
    s = 1 << level
    sl = tuple(slice(0, None, s) for _ in f.shape)
    idx = np.arange(f.size).reshape(f.shape)[sl].ravel()
    vals = f[sl].ravel()
    order = np.lexsort((idx, vals))
    return int(idx[order[0]]), int(idx[order[-1]])


@pytest.mark.parametrize("shape", [(2, 2, 2), (5, 3, 4), (3, 4, 5), (2, 9),
                                   (7, 6), (12, 10, 9)])
def test_linear_fields_have_two_critical_points(oracle_mod, shape):
    """A linear function on a convex triangulated domain has convex sublevel
    sets: one minimum, one maximum, nothing else.  Ties are broken by index,
    which keeps the order linear (value + eps * index)."""
    rng = np.random.default_rng(len(shape) * 100 + shape[0])
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    cases = [np.zeros(shape), grids[-1], grids[0]]
    for _ in range(4):
        coef = rng.integers(-3, 4, size=len(shape))
        cases.append(sum(c * g for c, g in zip(coef, grids)))
    for f in cases:
        f = np.ascontiguousarray(f, dtype=np.float32)
        for level in range(0, oracle_mod.max_level(shape) + 1):
            r = oracle_mod.classify(f, level=level)
            lo, hi = _argext(f, level)
            assert sorted(r.crit.tolist()) == sorted({lo, hi})
            flat = r.codes.ravel()
            assert flat[lo] & 7 == 0          # minimum: empty lower link
            assert (flat[hi] >> 3) & 7 == 0   # maximum: empty upper link


def test_constant_field_extremes_are_first_and_last(oracle_mod):
    f = np.zeros((6, 7, 8), np.float32)
    r = oracle_mod.classify(f)
    assert r.crit.tolist() == [0, f.size - 1]


@pytest.mark.parametrize("seed", range(6))
def test_separable_2d_product_of_1d(oracle_mod, seed):
    """f(x, y) = gx(x) + gy(y) with distinct integer values: an interior vertex
    is critical iff x is a 1D extremum of gx and y one of gy; max/max gives a
    maximum, min/min a minimum, mixed a saddle."""
    rng = np.random.default_rng(seed)
    nx, ny = 23 + seed, 17 + 2 * seed
    gx = rng.permutation(1000)[:nx].astype(np.int64)
    gy = rng.permutation(1000)[:ny].astype(np.int64) * 1000
    f = (gy[:, None] + gx[None, :]).astype(np.float32)
    assert np.array_equal(f.astype(np.int64), gy[:, None] + gx[None, :])

    def ext1d(g):
        out = np.zeros(len(g), np.int64)  # 1 = max, -1 = min, 0 = regular
        for i in range(1, len(g) - 1):
            if g[i] > g[i - 1] and g[i] > g[i + 1]:
                out[i] = 1
            elif g[i] < g[i - 1] and g[i] < g[i + 1]:
                out[i] = -1
        return out

    ex, ey = ext1d(gx), ext1d(gy)
    r = oracle_mod.classify(f)
    codes = r.codes
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            c = int(codes[y, x])
            nl, nu = c & 7, (c >> 3) & 7
            crit = not (nl == 1 and nu == 1)
            assert crit == bool(ex[x] and ey[y]), (x, y)
            if ex[x] == 1 and ey[y] == 1:
                assert nu == 0
            elif ex[x] == -1 and ey[y] == -1:
                assert nl == 0
            elif ex[x] and ey[y]:
                assert nl == 2 and nu == 2


# --------------------------------------------------------------------------
# Brute force on tiny grids
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(3, 3, 3), (2, 3, 4), (4, 2, 3), (4, 5),
                                   (3, 3)])
@pytest.mark.parametrize("seed", range(3))
def test_bruteforce_tiny(oracle_mod, shape, seed):
    """Every vertex of a tiny tie-heavy grid: component counts and Euler
    characteristics of both link parts, and chi(Lk-) against the Euler change
    of the sublevel complex counted over all simplices."""
    f = fieldgen.tie_field(shape, 10 + seed, 3)
    fx, sxyz = bf.field_xyz(f)
    cplx = bf.Complex(sxyz)
    pts = bf.grid_points(sxyz)
    coords = [p if len(p) == 3 else (p[0], p[1], 0) for p in pts]
    d = oracle_mod.vertex_detail(f, coords)
    total = 0
    for p, row in zip(pts, d):
        nl, nu, chil, chiu, dchi = cplx.vertex_stats(fx, p)
        assert (row[1], row[2], row[3], row[4]) == (nl, nu, chil, chiu), p
        assert 1 - chil == dchi
        total += dchi
        bl = bf.link_part_betti(cplx, fx, p, True)
        bu = bf.link_part_betti(cplx, fx, p, False)
        assert (row[5], row[6]) == (bl[1], bu[1]), p
        assert (bl[0], bu[0]) == (nl, nu)
        boundary = any(c in (0, n - 1) for c, n in zip(p, sxyz))
        assert row[8] == int(boundary and (bl[1] + bu[1] > 0))
        # regular (Section 3.1): both parts non-empty and simply connected;
        # these link parts are planar, so simply connected = b0 1 and b1 0
        regular = bl[:2] == (1, 0) and bu[:2] == (1, 0)
        assert row[9] == int(not regular), p
    assert total == 1


def test_boundary_annulus_is_critical(oracle_mod):
    """A vertex in the middle of a boundary face whose only upper neighbour
    is the link vertex straight inside: its lower link is an annulus --
    connected but not simply connected -- so it is critical although both
    link parts have one component (Section 3.1 asks for simple
    connectedness)."""
    f = np.full((2, 3, 3), -1.0, np.float32)   # (z, y, x); v = (1, 1, 0)
    f[0, 1, 1] = 0.0
    f[1, 1, 1] = 1.0
    fx, sxyz = bf.field_xyz(f)
    cplx = bf.Complex(sxyz)
    assert bf.link_part_betti(cplx, fx, (1, 1, 0), True)[:2] == (1, 1)
    row = oracle_mod.vertex_detail(f, [(1, 1, 0)])[0]
    assert (row[1], row[2], row[5], row[7], row[8], row[9]) == (1, 1, 1, 1, 1, 1)
    assert row[0] == 1 | (1 << 3) | (1 << 6) | (1 << 7)


# --------------------------------------------------------------------------
# Levels: level k is the sub-grid of stride 2^k
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(17, 12, 9), (33, 20), (9, 9, 9), (26, 7)])
def test_level_equals_subsampled_grid(oracle_mod, shape):
    """Restricted to a level, the index order is the level's own index order,
    so classifying level k equals classifying the subsampled array."""
    f = fieldgen.tie_field(shape, 5, 4)
    for level in range(1, oracle_mod.max_level(shape) + 1):
        s = 1 << level
        sub = np.ascontiguousarray(f[tuple(slice(0, None, s) for _ in shape)])
        a = oracle_mod.classify(f, level=level)
        b = oracle_mod.classify(sub, level=0)
        full_idx = np.arange(f.size).reshape(f.shape)[
            tuple(slice(0, None, s) for _ in shape)].ravel()
        assert np.array_equal(full_idx[b.crit.astype(np.int64)], a.crit)
        assert np.array_equal(
            a.codes[tuple(slice(0, None, s) for _ in shape)], b.codes)


def _window_planes(shape, level, a, b):
    """Full-resolution slow-axis positions of level-local planes [a, b)."""
    return np.arange(a, b) * (1 << level)


@pytest.mark.parametrize("shape", [(19, 14, 11), (13, 9, 20), (37, 23), (21, 40)])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_slow_range_window_equals_full_run(oracle_mod, shape, level):
    """Classification is local to a vertex's star (Section 3.1), so the
    windowed mode (level-local planes / rows [a, b) of the slowest axis) must
    give exactly the codes and list entries of the full-range run inside the
    window: windows at the low boundary, in the interior and at the high
    boundary."""
    f = fieldgen.tie_field(shape, 3 + level, 5)
    full = oracle_mod.classify(f, level=level)
    assert full.status == 0
    m = oracle_mod.level_dims(shape, level)
    n_slow = m[2] if len(shape) == 3 else m[1]
    s = 1 << level
    plane = int(np.prod(shape[1:]))  # full-resolution samples per slow step
    for a, b in [(0, 2), (1, n_slow - 1), (n_slow // 2, n_slow // 2 + 1),
                 (n_slow - 2, n_slow), (0, n_slow)]:
        w = oracle_mod.classify(f, level=level, slow_range=(a, b))
        assert w.status == 0
        # codes: every level position inside the window, none outside
        sel = [slice(0, None, s)] * len(shape)
        sel[0] = _window_planes(shape, level, a, b)
        assert np.array_equal(w.codes[tuple(sel)], full.codes[tuple(sel)])
        outside = np.ones(shape[0], bool)
        outside[_window_planes(shape, level, a, b)] = False
        assert not w.codes[outside].any()
        lo, hi = a * s * plane, (b - 1) * s * plane + plane
        inside = full.crit[(full.crit >= lo) & (full.crit < hi)]
        assert np.array_equal(w.crit, inside)
        assert w.count == len(inside)


@pytest.mark.parametrize("shape", [(17, 12, 9), (23, 15), (40, 7, 6)])
def test_window_of_sub_array_with_neighbour_planes(oracle_mod, shape):
    """The form the largest-grid GPU test uses: planes (rows) [a, b) are
    classified from the sub-array [a-1, b+1) clipped to the grid, and its
    indices, shifted by (a-1) planes, are the full run's.  Every window vertex
    keeps its whole star (one plane per side), and shifting all indices by a
    constant keeps their order."""
    f = fieldgen.iid_field(shape, 11)
    f[::3] = np.round(f[::3] * 4) / 4  # ties across planes
    full = oracle_mod.classify(f)
    n0 = shape[0]
    plane = int(np.prod(shape[1:]))
    for a, b in [(0, 3), (4, 9), (n0 - 3, n0), (0, n0), (1, 2)]:
        lo, hi = max(a - 1, 0), min(b + 1, n0)
        sub = np.ascontiguousarray(f[lo:hi])
        w = oracle_mod.classify(sub, slow_range=(a - lo, b - lo))
        assert w.status == 0
        assert np.array_equal(w.codes[a - lo:b - lo], full.codes[a:b])
        got = w.crit.astype(np.int64) + lo * plane
        exp = full.crit[(full.crit >= a * plane) & (full.crit < b * plane)]
        assert np.array_equal(got, exp.astype(np.int64))


def test_window_matches_bruteforce(oracle_mod):
    """Windowed classification of a tiny tie-heavy grid against the
    independent brute force (GF(2) Betti numbers of both link parts), vertex
    by vertex: a vertex is regular iff both parts have b0 = 1 and b1 = 0."""
    shape = (5, 4, 3)
    f = fieldgen.tie_field(shape, 9, 3)
    fx, sxyz = bf.field_xyz(f)
    cplx = bf.Complex(sxyz)
    for a, b in [(0, 1), (2, 4), (4, 5)]:
        w = oracle_mod.classify(f, slow_range=(a, b))
        for z in range(a, b):
            for y in range(shape[1]):
                for x in range(shape[2]):
                    bl = bf.link_part_betti(cplx, fx, (x, y, z), True)
                    bu = bf.link_part_betti(cplx, fx, (x, y, z), False)
                    regular = bl[:2] == (1, 0) and bu[:2] == (1, 0)
                    got = bool(oracle_mod.is_critical_code(w.codes[z, y, x]))
                    assert got == (not regular), (x, y, z)


def test_level_dims_and_max_level(oracle_mod):
    assert oracle_mod.level_dims((512, 512, 512), 8) == (2, 2, 2)
    assert oracle_mod.level_dims((512, 512, 512), 0) == (512, 512, 512)
    assert oracle_mod.level_dims((256, 256, 256), 7) == (2, 2, 2)
    assert oracle_mod.max_level((512, 512, 512)) == 8
    assert oracle_mod.max_level((256, 256, 256)) == 7
    assert oracle_mod.max_level((8192, 8192)) == 12
    assert oracle_mod.max_level((64, 64, 64)) == 5
    assert oracle_mod.level_dims((10, 6), 2) == (2, 3, 1)
    with pytest.raises(ValueError):
        oracle_mod.level_dims((5, 5, 5), 3)


# --------------------------------------------------------------------------
# i.i.d. statistics
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,p_ext", [((40, 40, 40), 1.0 / 15),
                                         ((300, 300), 1.0 / 7)])
def test_iid_extremum_probability(oracle_mod, shape, p_ext):
    """For i.i.d. continuous values an interior vertex is a minimum iff it is
    the smallest of itself and its neighbours: probability 1/(1 + #nbrs)."""
    f = fieldgen.iid_field(shape, 7)
    r = oracle_mod.classify(f)
    inner = r.codes[(slice(1, -1),) * len(shape)]
    n = inner.size
    for k in ((inner & 7) == 0, ((inner >> 3) & 7) == 0):
        frac = k.sum() / n
        sd = np.sqrt(p_ext * (1 - p_ext) / n)
        assert abs(frac - p_ext) < 5 * sd


# --------------------------------------------------------------------------
# Status codes
# --------------------------------------------------------------------------
def test_nan_and_capacity(oracle_mod):
    f = fieldgen.iid_field((6, 6, 6), 1)
    r = oracle_mod.classify(f, cap=3)
    assert r.status == oracle_mod.E_CAPACITY and r.count > 3
    assert len(r.crit) == 3
    full = oracle_mod.classify(f)
    assert np.array_equal(full.crit[:3], r.crit)
    f[2, 3, 4] = np.nan
    r = oracle_mod.classify(f)
    assert r.status == oracle_mod.E_NAN
