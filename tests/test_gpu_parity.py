"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results, so the bar is byte equality of the code array (at level
positions) and of the ascending critical list.  Cases: every interior
polarity pattern, every boundary class with every pattern of its present
neighbours, the 64^3 Gaussian workload, ragged and tie-heavy grids at every
level, the progressive driver per level, error paths, and the full-size
workloads on every vertex, plus the padded Morse count.
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
OFF2 = [(-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, 1)]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(dev):
    return pc.Context(0)


def gpu_classify(ctx, dev, f, level=0, **kw):
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    r = pc.classify(ft, level, ctx=ctx, **kw)
    torch.cuda.synchronize()
    return r


def level_mask(shape, level):
    s = 1 << level
    m = np.zeros(shape, bool)
    m[tuple(slice(0, None, s) for _ in shape)] = True
    return m


def assert_same(f, level, r, ref, what=""):
    codes = r.codes.cpu().numpy()
    lm = level_mask(f.shape, level)
    assert np.array_equal(codes[lm], ref.codes[lm]), f"codes differ {what}"
    crit = r.crit.cpu().numpy().view(np.uint32)
    assert np.array_equal(crit, ref.crit), f"list differs {what}"
    assert r.count == ref.count


# ---------------------------------------------------------------------------
# Exhaustive patterns
# ---------------------------------------------------------------------------
def test_all_interior_patterns(ctx, dev):
    bx, by, bz = 32, 32, 16
    f = np.full((3 * bz, 3 * by, 3 * bx), 0.25, np.float32)
    for b in range(1 << 14):
        cx, cy, cz = 3 * (b % bx) + 1, 3 * ((b // bx) % by) + 1, 3 * (b // (bx * by)) + 1
        f[cz, cy, cx] = 0.0
        for j, (dx, dy, dz) in enumerate(OFF3):
            f[cz + dz, cy + dy, cx + dx] = 1.0 if (b >> j) & 1 else -1.0
    log("interior patterns", f.shape)
    r = gpu_classify(ctx, dev, f)
    assert_same(f, 0, r, oracle.classify(f), "interior patterns")


def _boundary_classes(dim):
    """(side per axis) with at least one cut side: -1 low, +1 high, 0 free."""
    for sides in itertools.product((-1, 0, 1), repeat=dim):
        if any(sides):
            yield sides


def _boundary_grids(sides, offsets):
    """Grids placing every polarity pattern of the present neighbours at a
    vertex of boundary class `sides`.  Cut axes have 2 samples (the centre on
    the cut side), free axes pack patterns every 3 samples."""
    dim = len(sides)
    present = [j for j, o in enumerate(offsets)
               if all(not (s == -1 and d == -1) and not (s == 1 and d == 1)
                      for s, d in zip(sides, o))]
    npat = 1 << len(present)
    free = [a for a in range(dim) if sides[a] == 0]
    per_grid = npat if free else 1
    if len(free) == 2:
        side_len = [int(np.ceil(np.sqrt(npat)))] * 2
    elif len(free) == 1:
        side_len = [npat]
    else:
        side_len = []
    grids = []
    for g0 in range(0, npat, per_grid):
        ext = []
        fi = 0
        for a in range(dim):
            if sides[a] == 0:
                ext.append(3 * side_len[fi])
                fi += 1
            else:
                ext.append(2)
        f = np.full(tuple(reversed(ext)), 0.25, np.float32)  # C order
        for p in range(g0, min(npat, g0 + per_grid)):
            q = p - g0
            centre = []
            fi = 0
            for a in range(dim):
                if sides[a] == -1:
                    centre.append(0)
                elif sides[a] == 1:
                    centre.append(1)
                else:
                    if fi == 0:
                        centre.append(3 * (q % side_len[0]) + 1)
                    else:
                        centre.append(3 * (q // side_len[0]) + 1)
                    fi += 1
            f[tuple(reversed(centre))] = 0.0
            for bit, j in enumerate(present):
                nb = tuple(c + d for c, d in zip(centre, offsets[j]))
                f[tuple(reversed(nb))] = 1.0 if (p >> bit) & 1 else -1.0
        grids.append(f)
    return grids


@pytest.mark.parametrize("dim", [3, 2])
def test_all_boundary_patterns(ctx, dev, dim):
    offsets = OFF3 if dim == 3 else OFF2
    ncalls = 0
    for sides in _boundary_classes(dim):
        for f in _boundary_grids(sides, offsets):
            r = gpu_classify(ctx, dev, f)
            assert_same(f, 0, r, oracle.classify(f, threads=1), f"class {sides}")
            ncalls += 1
    log("boundary classes checked with", ncalls, "grids")


# ---------------------------------------------------------------------------
# Workloads and ragged grids, direct
# ---------------------------------------------------------------------------
def test_gauss64_direct(ctx, dev):
    f = fieldgen.config_field("gauss64")
    r = gpu_classify(ctx, dev, f, with_crit_codes=True)
    ref = oracle.classify(f)
    assert_same(f, 0, r, ref, "gauss64")
    cc = r.crit_codes.cpu().numpy()
    assert np.array_equal(cc, ref.codes.ravel()[ref.crit])


RAGGED = [(37, 23, 19), (3, 64, 65), (66, 5, 130), (2, 2, 2), (9, 2, 70),
          (19, 33, 129), (301, 77), (2, 1000), (1000, 2), (65, 257), (5, 5)]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("gen", ["tie", "gauss"])
def test_ragged_all_levels_direct(ctx, dev, shape, gen):
    f = (fieldgen.tie_field(shape, 3, 3) if gen == "tie" else
         fieldgen.gaussian_field(shape, 4, 5, noise=("uniform", 1e-3)))
    for level in range(pc.max_level(shape) + 1):
        r = gpu_classify(ctx, dev, f, level)
        assert_same(f, level, r, oracle.classify(f, level=level),
                    f"{shape} level {level}")


def test_special_values(ctx, dev):
    """+-inf are ordinary values; -0 equals +0 (ties go to the index)."""
    f = fieldgen.tie_field((11, 12, 13), 9, 4)
    vals = np.array([-np.inf, -0.0, 0.0, np.inf, 1.0], np.float32)
    f = vals[f.astype(np.int64) % 5].astype(np.float32)
    f.ravel()[::7] = -0.0
    r = gpu_classify(ctx, dev, f)
    assert_same(f, 0, r, oracle.classify(f), "special values")


def test_subnormal_values(ctx, dev):
    """Subnormal samples (a smooth field decaying into the subnormal range,
    mixed with exact ties and signed zeros): the sign of a difference of two
    subnormals must still decide the order."""
    rng = np.random.default_rng(5)
    tiny = np.float32(1.4e-45)  # smallest positive subnormal
    vals = np.array([0.0, -0.0, tiny, -tiny, 2 * tiny, 3e-40, -3e-40,
                     1.1e-38, 1.2e-38], np.float32)
    for shape in [(19, 21, 70), (67, 131)]:
        f = vals[rng.integers(0, len(vals), size=shape)]
        g = (rng.random(size=shape, dtype=np.float32) * np.float32(1e-39))
        f = np.where(rng.random(size=shape) < 0.5, f, g).astype(np.float32)
        assert (np.abs(f[f != 0]) < np.float32(1.18e-38)).any()
        r = gpu_classify(ctx, dev, f)
        assert_same(f, 0, r, oracle.classify(f), f"subnormal {shape}")
        check_progressive(ctx, dev, f)


def test_extreme_magnitudes(ctx, dev):
    """Samples near +-FLT_MAX, whose differences overflow to +-inf (the sign
    still carries the order), mixed with ordinary values and ties."""
    rng = np.random.default_rng(6)
    big = np.finfo(np.float32).max
    vals = np.array([big, -big, np.nextafter(big, 0, dtype=np.float32),
                     -np.nextafter(big, 0, dtype=np.float32), 1e38, -1e38,
                     0.0, 1.0, -1.0], np.float32)
    for shape in [(19, 21, 70), (67, 131)]:
        f = vals[rng.integers(0, len(vals), size=shape)].astype(np.float32)
        r = gpu_classify(ctx, dev, f)
        assert_same(f, 0, r, oracle.classify(f), f"extreme {shape}")
        check_progressive(ctx, dev, f)


# ---------------------------------------------------------------------------
# Progressive
# ---------------------------------------------------------------------------
def check_progressive(ctx, dev, f, per_level_oracle=True):
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    p = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    assert p.status == 0
    crit_all = p.crit.cpu().numpy().view(np.uint32)
    cc_all = p.crit_codes.cpu().numpy()
    for i, k in enumerate(p.levels):
        lst = crit_all[p.offsets[i]:p.offsets[i + 1]]
        if per_level_oracle:
            ref = oracle.classify(f, level=k)
            assert np.array_equal(lst, ref.crit), f"level {k} list"
            assert np.array_equal(cc_all[p.offsets[i]:p.offsets[i + 1]],
                                  ref.codes.ravel()[ref.crit]), f"level {k} codes"
    d = pc.classify(ft, 0, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(p.codes.cpu().numpy(), d.codes.cpu().numpy())
    assert np.array_equal(crit_all[p.offsets[-2]:p.offsets[-1]],
                          d.crit.cpu().numpy().view(np.uint32))
    return p


@pytest.mark.parametrize("shape", [(37, 23, 19), (33, 33, 33), (66, 5, 130),
                                   (2, 2, 2), (17, 9, 40), (301, 77), (2, 1000),
                                   (129, 130)])
@pytest.mark.parametrize("gen", ["tie", "gauss"])
def test_progressive_small(ctx, dev, shape, gen):
    f = (fieldgen.tie_field(shape, 5, 3) if gen == "tie" else
         fieldgen.gaussian_field(shape, 6, 7, noise=("uniform", 1e-3)))
    check_progressive(ctx, dev, f)


def test_progressive_gsin256(ctx, dev):
    f = fieldgen.config_field("gsin256")
    log("gsin256 progressive, per-level oracle")
    p = check_progressive(ctx, dev, f)
    ft = torch.from_numpy(f).to(dev)
    q = pc.progressive(ft, ctx=ctx, with_crit_codes=True, count_reclassified=True)
    torch.cuda.synchronize()
    assert np.array_equal(q.offsets, p.offsets)
    n = int(p.offsets[-1])
    assert torch.equal(q.crit[:n], p.crit[:n]) and torch.equal(q.codes, p.codes)
    assert torch.equal(q.crit_codes[:n], p.crit_codes[:n])
    assert q.reclassified[0] == 0
    assert (q.reclassified[1:] > 0).all()
    log("reclassified per level", q.reclassified.tolist())


def test_progressive_gauss64(ctx, dev):
    check_progressive(ctx, dev, fieldgen.config_field("gauss64"))


def _dirty_old_vertices(f, k):
    """Old vertices of level k (present at level k+1) whose neighbourhood
    changed: a neighbour direction present at one of the two levels only, or
    whose level-k neighbour v+d and level-(k+1) neighbour v+2d lie on
    different sides of v in the order (value, then full-resolution index).
    Counted directly on the level-k samples."""
    s = 1 << k
    offs = OFF3 if f.ndim == 3 else [(dx, dy, 0) for dx, dy in OFF2]
    f3 = f if f.ndim == 3 else f[None]
    lv = f3[::1 if f.ndim == 2 else s, ::s, ::s]
    nzf, nyf, nxf = f3.shape
    mz, my, mx = lv.shape
    zz, yy, xx = np.meshgrid(np.arange(mz), np.arange(my), np.arange(mx), indexing="ij")
    idx = (xx * s + nxf * (yy * s + nyf * (zz * (s if f.ndim == 3 else 1)))).astype(np.int64)
    old = (xx % 2 == 0) & (yy % 2 == 0) & (zz % 2 == 0)
    last = [2 * ((m - 1) // 2) for m in (mx, my, mz)]

    def after(a, b, ia, ib):  # a comes after b
        return (a > b) | ((a == b) & (ia > ib))

    dirty = np.zeros(lv.shape, bool)
    for dx, dy, dz in offs:
        x1, y1, z1 = xx + dx, yy + dy, zz + dz
        x2, y2, z2 = xx + 2 * dx, yy + 2 * dy, zz + 2 * dz
        e1 = (x1 >= 0) & (x1 < mx) & (y1 >= 0) & (y1 < my) & (z1 >= 0) & (z1 < mz)
        e2 = ((x2 >= 0) & (x2 <= last[0]) & (y2 >= 0) & (y2 <= last[1]) &
              (z2 >= 0) & (z2 <= last[2]))
        c1 = np.clip
        a1 = lv[c1(z1, 0, mz - 1), c1(y1, 0, my - 1), c1(x1, 0, mx - 1)]
        i1 = idx[c1(z1, 0, mz - 1), c1(y1, 0, my - 1), c1(x1, 0, mx - 1)]
        a2 = lv[c1(z2, 0, mz - 1), c1(y2, 0, my - 1), c1(x2, 0, mx - 1)]
        i2 = idx[c1(z2, 0, mz - 1), c1(y2, 0, my - 1), c1(x2, 0, mx - 1)]
        flip = after(a1, lv, i1, idx) != after(a2, lv, i2, idx)
        dirty |= (e1 != e2) | (e1 & e2 & flip)
    return int((dirty & old).sum())


@pytest.mark.parametrize("shape", [(37, 23, 19), (33, 33, 33), (17, 9, 40),
                                   (301, 77), (129, 130)])
@pytest.mark.parametrize("gen", ["tie", "gauss"])
def test_progressive_unfused_and_reclassified(ctx, dev, shape, gen):
    """A per-level callback makes every level a launch of its own (old
    vertices tested against stored masks); without it the small levels share
    one launch (masks recomputed from the field).  Both give the same lists,
    codes and re-classification counts, and the counts match a direct count
    of the old vertices whose neighbourhood changed."""
    f = (fieldgen.tie_field(shape, 7, 3) if gen == "tie" else
         fieldgen.gaussian_field(shape, 8, 6, noise=("uniform", 1e-3)))
    ft = torch.from_numpy(f).to(dev)
    seen = []
    p1 = pc.progressive(ft, ctx=ctx, with_crit_codes=True, count_reclassified=True,
                        callback=lambda k, n, u: seen.append((k, n)))
    torch.cuda.synchronize()
    p2 = pc.progressive(ft, ctx=ctx, with_crit_codes=True, count_reclassified=True)
    torch.cuda.synchronize()
    assert [k for k, _ in seen] == list(p1.levels)
    assert [n for _, n in seen] == list(np.diff(p1.offsets))
    assert np.array_equal(p1.offsets, p2.offsets)
    n = int(p1.offsets[-1])  # entries past the last list are not written
    assert torch.equal(p1.crit[:n], p2.crit[:n])
    assert torch.equal(p1.crit_codes[:n], p2.crit_codes[:n])
    assert torch.equal(p1.codes, p2.codes)
    assert np.array_equal(p1.reclassified, p2.reclassified)
    want = [0] + [_dirty_old_vertices(f, k) for k in p1.levels[1:]]
    assert list(p1.reclassified) == want
    check_progressive(ctx, dev, f)


@pytest.mark.parametrize("shape", [(130, 130, 257), (130, 132, 256)])
@pytest.mark.parametrize("callback", [False, True])
def test_progressive_without_list_codes(ctx, dev, shape, callback):
    """Without crit_codes only the last level stores full-resolution codes.
    Grids above 2^22 vertices give level 0 a launch of its own that reads the
    masks the coarser launch stored (level-1 rows of odd and even length, so
    both mask write-outs run; whole and partial 64-column tiles, so both code
    write-outs run).  Every level's list equals the direct classification of
    that level, and the codes equal the direct level-0 codes and the
    oracle's."""
    f = fieldgen.gaussian_field(shape, 16, 11, noise=("uniform", 1e-3))
    ft = torch.from_numpy(f).to(dev)
    log(f"progressive without list codes {shape} callback={callback}")
    cb = (lambda k, n, u: None) if callback else None
    p = pc.progressive(ft, ctx=ctx, callback=cb)
    torch.cuda.synchronize()
    assert p.status == 0 and p.crit_codes is None
    crit_all = p.crit.cpu().numpy().view(np.uint32)
    for i, k in enumerate(p.levels):
        d = pc.classify(ft, k, ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(crit_all[p.offsets[i]:p.offsets[i + 1]],
                              d.crit.cpu().numpy().view(np.uint32)), f"level {k}"
    ref = oracle.classify(f, level=0)
    codes = p.codes.cpu().numpy()
    assert np.array_equal(codes, ref.codes)
    assert np.array_equal(crit_all[p.offsets[-2]:p.offsets[-1]], ref.crit)


@pytest.mark.parametrize("shape", [(37, 23, 19), (130, 130, 257), (301, 77)])
def test_progressive_async_matches_sync(ctx, dev, shape):
    """The asynchronous call enqueues the same work: after several calls in
    a row (no host synchronisation between them) its device offsets, lists
    and codes equal the synchronous call's."""
    f = fieldgen.gaussian_field(shape, 16, 13, noise=("uniform", 1e-3))
    ft = torch.from_numpy(f).to(dev)
    log(f"progressive async {shape}")
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    codes, crit, offs = None, None, None
    for _ in range(3):
        codes, crit, offs = pc.progressive_async(ft, ctx=ctx, codes=codes, crit=crit,
                                                 offsets=offs)
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    assert np.array_equal(o, p.offsets)
    n = int(o[-1])
    assert torch.equal(crit[:n], p.crit[:n])
    assert torch.equal(codes, p.codes)


@pytest.mark.parametrize("shape", [(20, 21, 66), (130, 130, 257)])
def test_progressive_async_nan_and_capacity(ctx, dev, shape):
    """Small grids publish the offsets with a kernel of their own, grids
    whose level 0 has a launch of its own from the end of its compaction."""
    f = fieldgen.gaussian_field(shape, 8, 5, noise=("uniform", 1e-3))
    ft = torch.from_numpy(f).to(dev)
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    total = int(p.offsets[-1])
    cap = total // 2
    crit = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    _, crit, offs = pc.progressive_async(ft, ctx=ctx, capacity=cap, crit=crit)
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    assert np.array_equal(o, p.offsets) and o[-1] > cap
    assert torch.equal(crit, p.crit[:cap])
    g = f.copy()
    g[3, 4, 5] = np.nan
    gt = torch.from_numpy(g).to(dev)
    _, _, offs = pc.progressive_async(gt, ctx=ctx)
    torch.cuda.synchronize()
    assert int(offs[-1].item()) == -1


def test_progressive_special_values(ctx, dev):
    f = fieldgen.tie_field((21, 22, 23), 9, 4)
    vals = np.array([-np.inf, -0.0, 0.0, np.inf, 1.0], np.float32)
    f = vals[f.astype(np.int64) % 5].astype(np.float32)
    f.ravel()[::7] = -0.0
    check_progressive(ctx, dev, f)
    g = fieldgen.tie_field((45, 66), 9, 4)
    g = vals[g.astype(np.int64) % 5].astype(np.float32)
    check_progressive(ctx, dev, g)


def test_determinism(ctx, dev):
    f = fieldgen.tie_field((40, 50, 70), 1, 2)
    a = gpu_classify(ctx, dev, f)
    b = gpu_classify(ctx, dev, f)
    assert torch.equal(a.codes, b.codes) and torch.equal(a.crit, b.crit)


# ---------------------------------------------------------------------------
# Error paths
# ---------------------------------------------------------------------------
def test_nan_reported(ctx, dev):
    f = fieldgen.iid_field((20, 21, 22), 2)
    f[5, 6, 7] = np.nan
    ft = torch.from_numpy(f).to(dev)
    r = pc.classify(ft, ctx=ctx, check=False)
    assert r.status == pc.E_NAN
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    pc.classify(ft, ctx=ctx, count_dev=cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == -1
    # a NaN off the level is not a sample of that level
    g = fieldgen.iid_field((20, 21, 22), 2)
    g[5, 6, 7] = np.nan
    r = pc.classify(torch.from_numpy(g).to(dev), 1, ctx=ctx)
    assert r.status == 0
    p = pc.progressive(ft, ctx=ctx, check=False)
    assert p.status == pc.E_NAN


def test_capacity(ctx, dev):
    f = fieldgen.iid_field((30, 31, 32), 3)
    ref = oracle.classify(f)
    ft = torch.from_numpy(f).to(dev)
    cap = ref.count // 3
    r = pc.classify(ft, ctx=ctx, capacity=cap, check=False)
    assert r.status == pc.E_CAPACITY and r.count == ref.count
    assert np.array_equal(r.crit.cpu().numpy().view(np.uint32), ref.crit[:cap])
    assert np.array_equal(r.codes.cpu().numpy(), ref.codes)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    pc.classify(ft, ctx=ctx, capacity=cap, count_dev=cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == ref.count
    p = pc.progressive(ft, ctx=ctx, capacity=10, check=False)
    assert p.status == pc.E_CAPACITY


def test_bad_arguments(ctx, dev):
    import ctypes
    lib = pc.binding._load()
    f = torch.zeros((4, 5, 6), dtype=torch.float32, device=dev)
    codes = torch.zeros((4, 5, 6), dtype=torch.uint8, device=dev)
    crit = torch.zeros(200, dtype=torch.int32, device=dev)
    cnt = ctypes.c_int64(0)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())

    def call(field, nx, ny, nz, level, codes_p, crit_p, cap):
        return lib.pcrit_classify(ctx.handle, s, field, nx, ny, nz, level,
                                  codes_p, crit_p, None, cap, ctypes.byref(cnt),
                                  None)
    assert call(None, 6, 5, 4, 0, P(codes), P(crit), 200) == pc.E_ARG
    assert call(P(f), 6, 5, 4, 0, None, P(crit), 200) == pc.E_ARG
    assert call(P(f), 6, 5, 4, 0, P(codes), None, 200) == pc.E_ARG
    assert call(ctypes.c_void_p(f.data_ptr() + 2), 6, 5, 4, 0, P(codes), P(crit),
                200) == pc.E_ARG
    assert call(P(f), 6, 5, 4, 3, P(codes), P(crit), 200) == pc.E_LEVEL
    assert call(P(f), 6, 5, 4, -1, P(codes), P(crit), 200) == pc.E_LEVEL
    assert call(P(f), 1, 5, 4, 0, P(codes), P(crit), 200) == pc.E_DIMS
    assert call(P(f), 6, 5, 4, 0, P(codes), P(crit), -1) == pc.E_ARG
    assert call(P(f), 6, 5, 4, 0, P(codes), P(crit), 200) == 0


def test_binding_rejects_bad_buffers_on_device(ctx, dev):
    """Undersized or mistyped output buffers raise before any launch."""
    f = torch.zeros((6, 7, 8), dtype=torch.float32, device=dev)
    n = f.numel()
    cases = [
        dict(codes=torch.zeros(n - 1, dtype=torch.uint8, device=dev)),
        dict(codes=torch.zeros(n, dtype=torch.int32, device=dev)),
        dict(crit=torch.zeros(n - 1, dtype=torch.int32, device=dev), capacity=n),
        dict(crit=torch.zeros(n, dtype=torch.int64, device=dev)),
        dict(codes=torch.zeros(f.shape, dtype=torch.uint8)),
    ]
    for kw in cases:
        with pytest.raises(pc.PcritError) as e:
            pc.classify(f, ctx=ctx, **kw)
        assert e.value.status == pc.E_ARG
    with pytest.raises(pc.PcritError):
        pc.progressive(f, ctx=ctx, crit_codes=torch.zeros(3, dtype=torch.uint8, device=dev),
                       capacity=10)
    with pytest.raises(pc.PcritError):
        pc.progressive_async(f, ctx=ctx, offsets=torch.zeros(2, dtype=torch.int64, device=dev))
    # a short list without a capacity gets the list's length as capacity
    crit = torch.zeros(5, dtype=torch.int32, device=dev)
    g = torch.from_numpy(fieldgen.iid_field((6, 7, 8), 3)).to(dev)
    r = pc.classify(g, ctx=ctx, crit=crit)
    torch.cuda.synchronize()
    assert r.status == pc.E_CAPACITY and r.count > 5 and r.crit.numel() == 5


# ---------------------------------------------------------------------------
# Full-size workloads: every vertex, and the padded Morse count
# ---------------------------------------------------------------------------
def _morse_from_codes(codes_t, dim):
    h = torch.bincount(codes_t.reshape(-1).to(torch.int64), minlength=256).cpu().numpy()
    c = np.arange(256)
    nl, nu = c & 7, (c >> 3) & 7
    if dim == 3:
        w = (nl == 0).astype(np.int64) - (nu == 0) - np.maximum(nl - 1, 0) + np.maximum(nu - 1, 0)
    else:
        w = (nl == 0).astype(np.int64) + (nu == 0) - np.maximum(nl - 1, 0)
    return int((h * w).sum())


@pytest.mark.parametrize("name", ["noisy512", "noisy8192"])
def test_full_size(ctx, dev, name):
    """The full-size workloads, every vertex of every level against the
    oracle (its threaded run takes seconds), direct and progressive."""
    log("generating", name)
    f = fieldgen.config_field(name, device="cuda")
    ft = torch.from_numpy(f).to(dev)
    log("direct", name)
    r = pc.classify(ft, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    ref = oracle.classify(f)
    log("oracle done; critical fraction", ref.count / f.size)
    assert_same(f, 0, r, ref, name)
    ref_flat = ref.codes.ravel()
    assert np.array_equal(r.crit_codes[:r.count].cpu().numpy(), ref_flat[ref.crit])
    p = pc.progressive(ft, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    assert torch.equal(p.codes, r.codes)
    crit_all = p.crit.cpu().numpy().view(np.uint32)
    ccodes_all = p.crit_codes.cpu().numpy()
    for i, k in enumerate(p.levels):
        lref = ref if k == 0 else oracle.classify(f, level=k)
        a, b = p.offsets[i], p.offsets[i + 1]
        assert np.array_equal(crit_all[a:b], lref.crit), k
        # list codes of every level (level k's own classification)
        assert np.array_equal(ccodes_all[a:b], lref.codes.ravel()[lref.crit]), k
        if 0 < k <= 2:
            d = gpu_classify(ctx, dev, f, k)
            assert_same(f, k, d, lref, f"{name} level {k}")
    # the asynchronous entry point (the bench's) enqueues the same work
    codes_a, crit_a, offs_a = pc.progressive_async(ft, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(offs_a.cpu().numpy(), p.offsets)
    n = int(p.offsets[-1])
    assert torch.equal(crit_a[:n], p.crit[:n]) and torch.equal(codes_a, p.codes)
    del r, p, codes_a, crit_a
    # padded Morse count: with a +inf layer every original vertex is interior
    log("padded Morse count", name)
    pad = torch.nn.functional.pad(ft.unsqueeze(0), (1, 1, 1, 1) + ((1, 1) if f.ndim == 3 else ()),
                                  value=float("inf")).squeeze(0).contiguous()
    q = pc.classify(pad, ctx=ctx)
    torch.cuda.synchronize()
    inner = q.codes[(slice(1, -1),) * f.ndim]
    assert _morse_from_codes(inner, f.ndim) == 1


def test_repeated_direct_is_stable(ctx, dev):
    """Many z-chunks and blocks in flight: repeated direct passes give the
    same bytes as the progressive pass (which stages its planes differently)."""
    f = fieldgen.tie_field((200, 256, 320), 11, 3)
    ft = torch.from_numpy(f).to(dev)
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    for _ in range(5):
        r = pc.classify(ft, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(r.codes, p.codes)
        assert torch.equal(r.crit, p.level_list(0))
