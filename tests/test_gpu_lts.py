"""GPU parity of LTS Step 1 (superlevel / sublevel set propagation from
every extremum, Sections 4.2 and 4.5) against the oracle, through the C
ABI.  The GPU side takes its own order field and extremum lists (both
checked against the oracle's first); status, saddle and vertex count of
every propagation must equal the oracle's, for maxima and minima, several
epsilons and budgets, in 3D and 2D, with ties; the full-size noise field on
a sample of its extrema."""
import sys

import numpy as np
import pytest
import torch

import fieldgen
import oracle
from oracle import lts
from oracle.order import extrema as oracle_extrema, order_field as oracle_order
import paper_2009_00083_amd as pc

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(dev):
    return pc.Context(0)


def _gpu_inputs(ctx, dev, f):
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    rank, _ = pc.order_field(ft, ctx=ctx)
    codes = pc.classify(ft, ctx=ctx).codes
    mn, mx = pc.extrema(codes, ctx=ctx)
    torch.cuda.synchronize()
    return ft, rank, mn, mx


FIELDS = [
    ("gauss3d", lambda: fieldgen.gaussian_field((40, 36, 30), 31, 6, noise=("uniform", 2e-2))),
    ("iid3d", lambda: fieldgen.iid_field((24, 20, 18), 32)),
    ("ties3d", lambda: fieldgen.tie_field((22, 18, 16), 33, 3)),
    ("gauss2d", lambda: fieldgen.gaussian_field((120, 96), 34, 6, noise=("uniform", 2e-2))),
]


@pytest.mark.parametrize("name,make", FIELDS)
def test_matches_oracle(ctx, dev, name, make):
    f = make()
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    orank, _ = oracle_order(f)
    omn, omx = oracle_extrema(oracle.classify(f).codes)
    assert np.array_equal(rank.cpu().numpy().view(np.uint32), orank)
    assert np.array_equal(mn.cpu().numpy().view(np.uint32), omn)
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), omx)
    cases = [(np.inf, 16, 64), (0.0, 16, 64), (0.01, 16, 64), (0.05, 32, 128), (np.inf, 2, 14),
             (0.02, 5, 20)]
    for maxima in (True, False):
        ext, oext = (mx, omx) if maxima else (mn, omn)
        for eps, mv, mf in cases:
            st, sd, vi = pc.lts_propagate(ft, rank, ext, maxima=maxima, epsilon=eps,
                                          max_visited=mv, max_frontier=mf, ctx=ctx)
            torch.cuda.synchronize()
            ost, osd, ovi = lts.propagate_all(f, oext, eps, maxima=maxima, max_visited=mv,
                                              max_frontier=mf, rank=orank)
            what = (name, maxima, eps, mv, mf)
            assert np.array_equal(st.cpu().numpy(), ost), what
            assert np.array_equal(sd.cpu().numpy(), osd), what
            assert np.array_equal(vi.cpu().numpy().astype(np.uint16), ovi), what
            log(what, np.bincount(ost, minlength=3))


def test_full_size_sample(ctx, dev):
    """The 512^3 noise field: every maximum and minimum on the GPU; the
    oracle on 1500 of each, spread over the list."""
    f = fieldgen.config_field("noisy512", device="cuda")
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    orank = None
    for maxima, ext in ((True, mx), (False, mn)):
        st, sd, vi = pc.lts_propagate(ft, rank, ext, maxima=maxima, epsilon=0.05, ctx=ctx)
        torch.cuda.synchronize()
        n = ext.numel()
        pick = np.linspace(0, n - 1, 1500).astype(np.int64)
        if orank is None:
            orank = rank.cpu().numpy().view(np.uint32)  # checked against the oracle below
        e = ext.cpu().numpy().view(np.uint32)[pick]
        key = orank.astype(np.int64) if maxima else orank.size - 1 - orank.astype(np.int64)
        stc, sdc, vic = st.cpu().numpy()[pick], sd.cpu().numpy()[pick], vi.cpu().numpy()[pick]
        for j, m in enumerate(e):
            a, b, c = lts.propagate(f, key, f.shape, int(m), 0.05, 16, 64, maxima)
            assert (stc[j], sdc[j], vic[j]) == (a, b, c), (maxima, int(m))
        log("noisy512", "maxima" if maxima else "minima", n, np.bincount(st.cpu().numpy(), minlength=3))
    # the GPU order field on sampled vertices against the definition
    fl = f.ravel()
    idx = np.linspace(0, fl.size - 1, 16).astype(np.int64)
    for i in idx:
        below = np.count_nonzero(fl < fl[i]) + np.count_nonzero(fl[:i] == fl[i])
        assert orank[i] == below


def test_invalid_entries_and_arguments(ctx, dev):
    f = fieldgen.iid_field((12, 10, 8), 41)
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    bad = torch.tensor([int(mx[0]), f.size, f.size + 7, int(mx[-1])], dtype=torch.int32, device=dev)
    st, sd, vi = pc.lts_propagate(ft, rank, bad, ctx=ctx)
    torch.cuda.synchronize()
    assert st.cpu().tolist()[1:3] == [pc.LTS_INVALID, pc.LTS_INVALID]
    assert sd.cpu().tolist()[1:3] == [-1, -1]
    ref = lts.propagate_all(f, np.array([int(mx[0]), int(mx[-1])]), np.inf)
    assert [int(st[0]), int(st[3])] == list(ref[0])
    for kw in ({"max_visited": 1}, {"max_visited": pc.LTS_MAX_VISITED + 1},
               {"max_frontier": 13}, {"max_frontier": pc.LTS_MAX_FRONTIER + 1},
               {"epsilon": float("nan")}):
        with pytest.raises(pc.PcritError) as e:
            pc.lts_propagate(ft, rank, mx, ctx=ctx, **kw)
        assert e.value.status == pc.E_ARG
    empty = torch.empty(0, dtype=torch.int32, device=dev)
    st, sd, vi = pc.lts_propagate(ft, rank, empty, ctx=ctx)
    assert st.numel() == 0


# ---------------------------------------------------------------------------
# merged propagations (Sections 4.4 and 4.5)

MERGED_CASES = [(np.inf, 16, 64), (0.0, 16, 64), (0.01, 16, 64), (0.05, 32, 128),
                (np.inf, 2, 14), (0.02, 5, 20), (0.1, 32, 128), (np.inf, 32, 128)]


@pytest.mark.parametrize("name,make", FIELDS)
def test_merged_matches_oracle(ctx, dev, name, make):
    f = make()
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    orank, _ = oracle_order(f)
    omn, omx = oracle_extrema(oracle.classify(f).codes)
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), omx)
    assert np.array_equal(mn.cpu().numpy().view(np.uint32), omn)
    merged = 0
    for maxima in (True, False):
        ext, oext = (mx, omx) if maxima else (mn, omn)
        for eps, mv, mf in MERGED_CASES:
            st, sd, vi = pc.lts_merged(ft, rank, ext, maxima=maxima, epsilon=eps,
                                       max_visited=mv, max_frontier=mf, ctx=ctx)
            torch.cuda.synchronize()
            ost, osd, ovi = lts.propagate_merged(f, oext, eps, maxima, mv, mf, rank=orank)
            what = (name, maxima, eps, mv, mf)
            assert np.array_equal(st.cpu().numpy(), ost), what
            assert np.array_equal(sd.cpu().numpy(), osd), what
            assert np.array_equal(vi.cpu().numpy().astype(np.uint16), ovi), what
            ind = lts.propagate_all(f, oext, eps, maxima, mv, mf, rank=orank)
            merged += int(np.count_nonzero(ind[0] != ost))
            log("merged", what, np.bincount(ost, minlength=3))
    assert merged > 0  # some propagations went on past a saddle


def test_merged_noise_cube(ctx, dev):
    """A 96^3 noisy field: every maximum and minimum against the oracle, and
    a second GPU run identical to the first (arrival order varies)."""
    f = fieldgen.gaussian_field((96, 96, 96), 51, 6, noise=("uniform", 2e-2))
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    orank, _ = oracle_order(f)
    omn, omx = oracle_extrema(oracle.classify(f).codes)
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), omx)
    for maxima, ext, oext in ((True, mx, omx), (False, mn, omn)):
        runs = []
        for _ in range(2):
            st, sd, vi = pc.lts_merged(ft, rank, ext, maxima=maxima, epsilon=0.03, ctx=ctx)
            torch.cuda.synchronize()
            runs.append((st.cpu().numpy(), sd.cpu().numpy(), vi.cpu().numpy().astype(np.uint16)))
        log("merged cube", maxima, len(oext))
        ref = lts.propagate_merged(f, oext, 0.03, maxima, 16, 64, rank=orank)
        for run in runs:
            for a, b in zip(run, ref):
                assert np.array_equal(a, b), maxima


def test_merged_full_size_properties(ctx, dev):
    """The 512^3 noise field, every maximum and minimum: two GPU runs agree;
    a propagation that the independent one ends before its first saddle
    (persistent or budget) ends the same way merged; every removed extremum
    lies within epsilon of its saddle; on a sample of them the component is
    the strict superlevel (sublevel) component of the saddle plus the
    saddle, led by the extremum, and the saddle has a larger (smaller)
    neighbour outside it."""
    f = fieldgen.config_field("noisy512", device="cuda")
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    orank = rank.cpu().numpy().view(np.uint32)
    fl = f.ravel()
    eps = 0.05
    for maxima, ext in ((True, mx), (False, mn)):
        a = [t.cpu().numpy() for t in pc.lts_merged(ft, rank, ext, maxima=maxima, epsilon=eps, ctx=ctx)]
        b = [t.cpu().numpy() for t in pc.lts_merged(ft, rank, ext, maxima=maxima, epsilon=eps, ctx=ctx)]
        ind = [t.cpu().numpy() for t in pc.lts_propagate(ft, rank, ext, maxima=maxima, epsilon=eps, ctx=ctx)]
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
        st, sd, vi = a
        early = ind[0] != lts.SADDLE
        assert np.array_equal(st[early], ind[0][early]) and np.array_equal(vi[early], ind[2][early])
        e = ext.cpu().numpy().view(np.uint32).astype(np.int64)
        rem = np.flatnonzero(st == lts.SADDLE)
        d = (fl[e[rem]] - fl[sd[rem]]) if maxima else (fl[sd[rem]] - fl[e[rem]])
        assert np.all(d.astype(np.float32) <= np.float32(eps))
        log("merged noisy512", "maxima" if maxima else "minima", len(e), np.bincount(st, minlength=3),
            "differ from independent", int(np.count_nonzero(st != ind[0])))
        key = orank.astype(np.int64) if maxima else orank.size - 1 - orank.astype(np.int64)
        for j in rem[np.linspace(0, len(rem) - 1, 300).astype(np.int64)]:
            m, s = int(e[j]), int(sd[j])
            comp = lts.superlevel_component(f.shape, key, m, key[s] + 1)
            assert len(comp) + 1 == vi[j] and max(key[c] for c in comp) == key[m]
            assert any(u not in comp and key[u] > key[s] for u in lts.neighbours(f.shape, s))


def test_merged_invalid_entries_and_arguments(ctx, dev):
    f = fieldgen.iid_field((12, 10, 8), 41)
    ft, rank, mn, mx = _gpu_inputs(ctx, dev, f)
    notmax = int(mn[0])
    bad = torch.tensor([int(mx[0]), f.size, notmax, int(mx[-1])], dtype=torch.int32, device=dev)
    st, sd, vi = pc.lts_merged(ft, rank, bad, epsilon=0.1, ctx=ctx)
    torch.cuda.synchronize()
    ref = lts.propagate_merged(f, bad.cpu().numpy().view(np.uint32), 0.1)
    assert np.array_equal(st.cpu().numpy(), ref[0]) and np.array_equal(sd.cpu().numpy(), ref[1])
    assert st.cpu().tolist()[1:3] == [pc.LTS_INVALID, pc.LTS_INVALID]
    for kw in ({"max_visited": 1}, {"max_visited": pc.LTS_MAX_VISITED + 1},
               {"max_frontier": 13}, {"max_frontier": pc.LTS_MAX_FRONTIER + 1},
               {"epsilon": float("nan")}):
        with pytest.raises(pc.PcritError) as e:
            pc.lts_merged(ft, rank, mx, ctx=ctx, **kw)
        assert e.value.status == pc.E_ARG
    empty = torch.empty(0, dtype=torch.int32, device=dev)
    st, sd, vi = pc.lts_merged(ft, rank, empty, ctx=ctx)
    assert st.numel() == 0
