"""GPU parity at the largest grids the boundary accepts: N just below 2^32
vertices, so vertex indices and list positions pass 2^31 and level lists
are addressed with 64-bit offsets.

The oracle cannot classify 4.3 G vertices in a test's time, so it checks
windows of planes (3D) or rows (2D): one that straddles index 2^31 and the
last ones (the top boundary), each classified from the window plus one
neighbouring plane or row per side, which gives every vertex of the window
its full neighbourhood.  Whole-field properties cover the rest: the list is
strictly ascending, its length equals the number of critical codes, and the
progressive driver's level-0 and level-1 lists and codes equal the direct
passes', and the fractions of interior minima and maxima of the i.i.d. field
match their exact probability 1/(1 + neighbours) to sampling error.
"""
import numpy as np
import pytest
import torch

import fieldgen
import oracle
import paper_2009_00083_amd as pc

pytestmark = pytest.mark.gpu

CH = 1 << 28  # elements per chunk of the whole-field checks


def log(*a):
    print(*a, flush=True)


def _u32(t):
    return t.to(torch.int64) & 0xFFFFFFFF


def _count_below(crit, n, bound):
    """Entries of the ascending list crit[:n] (uint32 values) below bound."""
    tot = 0
    for s in range(0, n, CH):
        tot += int((_u32(crit[s:min(n, s + CH)]) < bound).sum())
    return tot


def _check_ascending(crit, n):
    prev = -1
    for s in range(0, n, CH):
        c = _u32(crit[s:min(n, s + CH)])
        assert int(c[0]) > prev
        assert bool((c[1:] > c[:-1]).all())
        prev = int(c[-1])


def _critical_codes(codes):
    flat = codes.reshape(-1)
    tot = 0
    for s in range(0, flat.numel(), CH):
        tot += int(((flat[s:s + CH] & 0xBF) != 9).sum())
    return tot


def _interior_extrema(codes):
    """(minima, maxima, vertices) over the interior vertices."""
    nmin = nmax = 0
    inner = codes[(slice(1, -1),) * codes.dim()]
    step = max(1, CH // max(1, inner[0].numel()))
    for s in range(0, inner.shape[0], step):
        c = inner[s:s + step]
        nmin += int(((c & 7) == 0).sum())
        nmax += int(((c & 0x38) == 0).sum())
    return nmin, nmax, inner.numel()


def _check_window(ft, codes, crit, n, a, b):
    """Codes and list entries of planes (rows) [a, b) against the oracle."""
    n0 = ft.shape[0]
    lo, hi = max(a - 1, 0), min(b + 1, n0)
    sub = ft[lo:hi].cpu().numpy()
    ref = oracle.classify(sub, slow_range=(a - lo, b - lo))
    assert ref.status == 0
    P = int(np.prod(ft.shape[1:]))
    assert np.array_equal(codes[a:b].cpu().numpy(), ref.codes[a - lo:b - lo])
    start = _count_below(crit, n, a * P)
    k = int(ref.count)
    got = crit[start:start + k].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(got, ref.crit.astype(np.int64) + lo * P)
    if start + k < n:
        assert int(_u32(crit[start + k:start + k + 1])) >= b * P
    return k


@pytest.mark.parametrize("shape,windows", [
    ((1023, 2048, 2048), [(511, 514), (1019, 1023)]),
    ((65535, 65535), [(32760, 32780), (65500, 65535)]),
])
def test_max_size(shape, windows):
    n_all = int(np.prod(shape))
    assert (1 << 31) < n_all < (1 << 32)
    dev = torch.device("cuda:0")
    ctx = pc.Context(0)
    log("max size", shape)
    ft = fieldgen.device_iid_field(shape, 21, dev)
    r = pc.classify(ft, ctx=ctx)
    torch.cuda.synchronize()
    n = r.count
    log("critical", n, "of", n_all)
    assert n == _critical_codes(r.codes)
    _check_ascending(r.crit, n)
    assert int(_u32(r.crit[n - 1:n])) >= 1 << 31
    # i.i.d. samples: an interior vertex is a minimum (maximum) iff it is
    # the smallest (largest) of itself and its 14 (6) neighbours
    p_ext = 1.0 / (15 if len(shape) == 3 else 7)
    nmin, nmax, ni = _interior_extrema(r.codes)
    sd = np.sqrt(p_ext * (1 - p_ext) / ni)
    log("extremum fractions", nmin / ni, nmax / ni, "expected", p_ext)
    assert abs(nmin / ni - p_ext) < 5 * sd and abs(nmax / ni - p_ext) < 5 * sd
    for a, b in windows:
        log("window", a, b)
        assert _check_window(ft, r.codes, r.crit, n, a, b) > 0
    log("progressive")
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    assert p.status == 0
    assert np.all(np.diff(p.offsets) >= 0)
    assert torch.equal(p.codes, r.codes)
    l0 = p.level_list(0)
    assert l0.numel() == n and torch.equal(l0, r.crit)
    del r
    r1 = pc.classify(ft, 1, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(p.level_list(1), r1.crit)
    del p, r1, ft
    ctx.close()
    torch.cuda.empty_cache()


def _check_window_mid(ft, codes, crit, n, a, b):
    """Codes and list entries of the index range [a, b) of the middle axis
    (rows of a two-plane 3D grid, columns of a two-row 2D grid) against the
    oracle, which classifies that range plus one neighbour per side.  The
    sub-grid keeps the lexicographic order of the vertices, so the tie-break
    is the same; its extra rows (columns) are not compared."""
    three = ft.dim() == 3
    lo, hi = max(a - 1, 0), min(b + 1, ft.shape[-2] if three else ft.shape[-1])
    sub = (ft[:, lo:hi, :] if three else ft[:, lo:hi]).contiguous().cpu().numpy()
    ref = oracle.classify(sub)
    assert ref.status == 0
    got_codes = (codes[:, a:b, :] if three else codes[:, a:b]).cpu().numpy()
    want_codes = ref.codes[:, a - lo:b - lo, :] if three else ref.codes[:, a - lo:b - lo]
    assert np.array_equal(got_codes, want_codes)
    # list entries: one run per plane (3D) or row (2D)
    nx = ft.shape[-1]
    outer = ft.shape[0]
    inner = ft.shape[1] * nx if three else nx        # vertices per plane / row
    unit = nx if three else 1                         # index step of the middle axis
    sub_inner = (hi - lo) * unit
    ref_idx = ref.crit.astype(np.int64)
    total = 0
    for o in range(outer):
        g0, g1 = o * inner + a * unit, o * inner + b * unit
        start = _count_below(crit, n, g0)
        stop = _count_below(crit, n, g1)
        got = crit[start:stop].cpu().numpy().view(np.uint32).astype(np.int64)
        s0, s1 = o * sub_inner + (a - lo) * unit, o * sub_inner + (b - lo) * unit
        sel = ref_idx[(ref_idx >= s0) & (ref_idx < s1)]
        want = sel - o * sub_inner - (a - lo) * unit + g0
        assert np.array_equal(got, want)
        total += len(got)
    return total


@pytest.mark.parametrize("shape,windows", [
    # planes of 2^30 - 4 vertices (the byte range of a buffer descriptor
    # ends at 2^32 - 1), 24940 = 4 * 5 * 29 * 43 columns (the quad tiles) by
    # 43053 = 3 * 113 * 127 rows; the last window ends at the last vertex
    ((2, 43053, 24940), [(21520, 21530), (43045, 43053)]),
    # a 2D row of 2^30 - 1 vertices, the largest accepted
    ((2, (1 << 30) - 1), [(1 << 29, (1 << 29) + 4096), ((1 << 30) - 4097, (1 << 30) - 1)]),
])
def test_plane_and_row_limit(shape, windows):
    n_all = int(np.prod(shape))
    assert n_all > (1 << 31) - (1 << 17)
    dev = torch.device("cuda:0")
    ctx = pc.Context(0)
    log("plane / row limit", shape)
    ft = fieldgen.device_iid_field(shape, 23, dev)
    r = pc.classify(ft, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    n = r.count
    log("critical", n, "of", n_all)
    assert n == _critical_codes(r.codes)
    _check_ascending(r.crit, n)
    assert int(_u32(r.crit[n - 1:n])) >= n_all - (1 << 16)
    for s in range(0, n, CH):
        idx = _u32(r.crit[s:min(n, s + CH)])
        want = r.codes.reshape(-1)[idx]
        assert torch.equal(r.crit_codes[s:min(n, s + CH)], want)
    for a, b in windows:
        log("window", a, b)
        assert _check_window_mid(ft, r.codes, r.crit, n, a, b) > 0
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    assert p.status == 0 and p.levels == [0]
    assert torch.equal(p.codes, r.codes)
    assert torch.equal(p.level_list(0), r.crit[:n])
    del r, p, ft
    ctx.close()
    torch.cuda.empty_cache()
