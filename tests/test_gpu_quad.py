"""GPU parity of the quad-tile kernels (full-resolution and stride-2 levels
of 3D grids whose rows start on 16-byte boundaries, i.e. nx % 4 == 0 at
level 0 and nx even at level 1) against the oracle, and of the other kernels
on the same inputs shifted off that alignment.

Every check goes through the C ABI and compares codes at every level vertex
and the ascending critical list byte for byte.
"""
import itertools
import sys

import numpy as np
import pytest
import torch

import fieldgen
import oracle
import paper_2009_00083_amd as pc

pytestmark = pytest.mark.gpu

OFF3 = [(0, 0, -1), (-1, 0, -1), (0, -1, -1), (-1, -1, -1),
        (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (-1, -1, 0), (1, 1, 0),
        (0, 0, 1), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(dev):
    return pc.Context(0)


def level_mask(shape, level):
    s = 1 << level
    m = np.zeros(shape, bool)
    m[tuple(slice(0, None, s) for _ in shape)] = True
    return m


def check(ctx, dev, f, level, what, with_codes=False):
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    r = pc.classify(ft, level, ctx=ctx, with_crit_codes=with_codes)
    torch.cuda.synchronize()
    ref = oracle.classify(f, level=level)
    codes = r.codes.cpu().numpy()
    lm = level_mask(f.shape, level)
    bad = np.flatnonzero((codes != ref.codes) & lm)
    assert bad.size == 0, f"{what}: {bad.size} codes differ, first at {bad[:5]}"
    crit = r.crit.cpu().numpy().view(np.uint32)
    assert np.array_equal(crit, ref.crit), f"{what}: list differs"
    if with_codes:
        assert np.array_equal(r.crit_codes.cpu().numpy(), ref.codes.ravel()[ref.crit])
    return r


def _interior_patterns():
    bx, by, bz = 32, 32, 16
    f = np.full((3 * bz, 3 * by, 3 * bx), 0.25, np.float32)
    for b in range(1 << 14):
        cx, cy, cz = 3 * (b % bx) + 1, 3 * ((b // bx) % by) + 1, 3 * (b // (bx * by)) + 1
        f[cz, cy, cx] = 0.0
        for j, (dx, dy, dz) in enumerate(OFF3):
            f[cz + dz, cy + dy, cx + dx] = 1.0 if (b >> j) & 1 else -1.0
    return f


@pytest.mark.parametrize("pad", [0, 1, 4])
def test_interior_patterns_both_kernels(ctx, dev, pad):
    """All 16384 interior polarity patterns; nx = 96 and 100 take the quad
    tiles, nx = 97 the other kernel."""
    f = _interior_patterns()
    if pad:
        f = np.concatenate([f, np.full(f.shape[:2] + (pad,), 0.5, np.float32)], axis=2)
    log("interior patterns", f.shape)
    check(ctx, dev, f, 0, f"interior patterns nx={f.shape[2]}")


def test_interior_patterns_level1(ctx, dev):
    """The same patterns at stride 2: the level-1 samples are the patterns,
    the samples in between are noise that level 1 must not read."""
    f = _interior_patterns()
    nz, ny, nx = f.shape
    g = np.random.default_rng(1).random((2 * nz - 1, 2 * ny - 1, 2 * nx), dtype=np.float32)
    g[::2, ::2, ::2] = f
    log("interior patterns at level 1", g.shape)
    r = check(ctx, dev, g, 1, "interior patterns level 1")
    direct = check(ctx, dev, f, 0, "interior patterns level 0")
    assert np.array_equal(r.codes.cpu().numpy()[::2, ::2, ::2], direct.codes.cpu().numpy())


def _boundary_grids(sides):
    """Every polarity pattern of the present neighbours at a vertex of
    boundary class `sides` (side per axis: -1 low, +1 high, 0 free), padded
    along x to a multiple of 4 samples without changing the class."""
    present = [j for j, o in enumerate(OFF3)
               if all(not (s == -1 and d == -1) and not (s == 1 and d == 1)
                      for s, d in zip(sides, o))]
    npat = 1 << len(present)
    free = [a for a in range(3) if sides[a] == 0]
    per_grid = npat if free else 1
    side_len = ([int(np.ceil(np.sqrt(npat)))] * 2 if len(free) == 2 else
                [npat] if len(free) == 1 else [])
    for g0 in range(0, npat, per_grid):
        ext, fi = [], 0
        for a in range(3):
            if sides[a] == 0:
                ext.append(3 * side_len[fi])
                fi += 1
            else:
                ext.append(2)
        f = np.full(tuple(reversed(ext)), 0.25, np.float32)
        for p in range(g0, min(npat, g0 + per_grid)):
            q = p - g0
            centre, fi = [], 0
            for a in range(3):
                if sides[a] == -1:
                    centre.append(0)
                elif sides[a] == 1:
                    centre.append(1)
                else:
                    centre.append(3 * (q % side_len[0]) + 1 if fi == 0 else
                                  3 * (q // side_len[0]) + 1)
                    fi += 1
            f[tuple(reversed(centre))] = 0.0
            for bit, j in enumerate(present):
                nb = tuple(c + d for c, d in zip(centre, OFF3[j]))
                f[tuple(reversed(nb))] = 1.0 if (p >> bit) & 1 else -1.0
        nx = f.shape[2]
        padn = (-nx) % 4 if nx > 2 else 2
        filler = np.full(f.shape[:2] + (padn,), 0.75, np.float32)
        if sides[0] == 1:  # keep the centre on the last column
            f = np.concatenate([filler, f], axis=2)
        elif padn:
            f = np.concatenate([f, filler], axis=2)
        yield f


def test_boundary_patterns_quad(ctx, dev):
    """All 26 boundary classes of 3D, each with every pattern of its present
    neighbours, on grids whose rows take the quad tiles."""
    n = 0
    for sides in itertools.product((-1, 0, 1), repeat=3):
        if not any(sides):
            continue
        for f in _boundary_grids(sides):
            assert f.shape[2] % 4 == 0
            check(ctx, dev, f, 0, f"class {sides} {f.shape}")
            n += 1
    log("boundary grids checked:", n)


QUAD_SHAPES = [(20, 37, 260), (9, 10, 516), (33, 45, 64), (40, 23, 256),
               (5, 6, 8), (3, 3, 4), (2, 2, 4), (17, 130, 132), (4, 3, 1028),
               (70, 2, 12), (2, 70, 20)]


@pytest.mark.parametrize("shape", QUAD_SHAPES)
@pytest.mark.parametrize("gen", ["tie", "gauss"])
def test_quad_ragged_all_levels(ctx, dev, shape, gen):
    """Ragged tiles in x (partial lanes), y (rows past the grid) and z
    (short last chunk), every level (0 and 1 on the quad tiles)."""
    f = (fieldgen.tie_field(shape, 13, 3) if gen == "tie" else
         fieldgen.gaussian_field(shape, 14, 5, noise=("uniform", 1e-3)))
    for level in range(pc.max_level(shape) + 1):
        check(ctx, dev, f, level, f"{shape} {gen} level {level}", with_codes=level < 2)


def _special_field(shape, seed):
    """Ties, signed zeros next to each other, infinities next to each other,
    subnormals and values near FLT_MAX."""
    rng = np.random.default_rng(seed)
    big = np.finfo(np.float32).max
    tiny = np.float32(1.4e-45)
    vals = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, tiny, -tiny, 3e-40,
                     big, -big, 0.5], np.float32)
    f = vals[rng.integers(0, len(vals), size=shape)]
    f[..., 1::5] = -0.0
    f[..., 2::5] = 0.0
    f[..., 3::7] = np.inf
    f[1::3, ..., 4::7] = np.inf
    return f.astype(np.float32)


@pytest.mark.parametrize("shape", [(11, 12, 16), (9, 7, 264), (6, 70, 8)])
def test_quad_special_values(ctx, dev, shape):
    f = _special_field(shape, sum(shape))
    for level in range(min(2, pc.max_level(shape) + 1)):
        check(ctx, dev, f, level, f"special {shape} level {level}", with_codes=True)


def test_quad_special_progressive(ctx, dev):
    f = _special_field((20, 33, 68), 3)
    ft = torch.from_numpy(f).to(dev)
    p = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    crit = p.crit.cpu().numpy().view(np.uint32)
    for i, k in enumerate(p.levels):
        ref = oracle.classify(f, level=k)
        assert np.array_equal(crit[p.offsets[i]:p.offsets[i + 1]], ref.crit), k


def test_quad_nan(ctx, dev):
    """A NaN on the level is reported; a NaN between level-1 samples is not
    read at level 1."""
    f = fieldgen.iid_field((10, 12, 40), 4)
    g = f.copy()
    g[4, 6, 20] = np.nan  # a level-1 sample
    ft = torch.from_numpy(g).to(dev)
    for level in (0, 1):
        r = pc.classify(ft, level, ctx=ctx, check=False)
        assert r.status == pc.E_NAN, level
    h = f.copy()
    h[4, 6, 21] = np.nan  # odd column: not a level-1 sample
    ft = torch.from_numpy(h).to(dev)
    assert pc.classify(ft, 0, ctx=ctx, check=False).status == pc.E_NAN
    r2 = pc.classify(ft, 1, ctx=ctx, check=False)
    assert r2.status == 0
    ref = oracle.classify(f, level=1)
    assert np.array_equal(r2.crit.cpu().numpy().view(np.uint32), ref.crit)


@pytest.mark.parametrize("shape", [(130, 132, 256), (66, 64, 132)])
def test_quad_progressive_modes_agree(ctx, dev, shape):
    """The progressive call with and without the re-classification count
    (which keeps level 0 and 1 off the quad tiles) gives the same lists and
    codes, equal to the oracle at every level."""
    f = fieldgen.gaussian_field(shape, 21, 9, noise=("uniform", 1e-3))
    ft = torch.from_numpy(f).to(dev)
    a = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    b = pc.progressive(ft, ctx=ctx, with_crit_codes=True, count_reclassified=True)
    torch.cuda.synchronize()
    assert np.array_equal(a.offsets, b.offsets)
    n = int(a.offsets[-1])
    assert torch.equal(a.crit[:n], b.crit[:n])
    assert torch.equal(a.crit_codes[:n], b.crit_codes[:n])
    assert torch.equal(a.codes, b.codes)
    crit = a.crit.cpu().numpy().view(np.uint32)
    for i, k in enumerate(a.levels):
        ref = oracle.classify(f, level=k)
        assert np.array_equal(crit[a.offsets[i]:a.offsets[i + 1]], ref.crit), k


def test_quad_misaligned_field_takes_other_kernel(ctx, dev):
    """A field view that starts 4 bytes into its buffer cannot use 16-byte
    loads; the result is the same."""
    f = fieldgen.gaussian_field((12, 20, 64), 2, 4, noise=("uniform", 1e-3))
    base = torch.zeros(f.size + 1, dtype=torch.float32, device=dev)
    base[1:] = torch.from_numpy(f.ravel()).to(dev)
    view = base[1:].view(f.shape)
    assert view.data_ptr() % 16 == 4
    r = pc.classify(view, 0, ctx=ctx)
    torch.cuda.synchronize()
    ref = oracle.classify(f)
    assert np.array_equal(r.crit.cpu().numpy().view(np.uint32), ref.crit)
    assert np.array_equal(r.codes.cpu().numpy(), ref.codes)
