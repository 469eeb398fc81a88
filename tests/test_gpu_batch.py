"""GPU parity of the batched classification (many independent fields, shared
launches) against the oracle field by field, and against the single-field
entry point byte for byte; capacity and NaN behaviour."""
import sys

import numpy as np
import pytest
import torch

import fieldgen
import oracle
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


def _fields(seed, n, dim, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(lo, hi + 1, size=dim))
        kind = i % 3
        if kind == 0:
            f = fieldgen.gaussian_field(shape, seed + i, 6, noise=("uniform", 1e-3))
        elif kind == 1:
            f = fieldgen.tie_field(shape, seed + i, 3)
        else:
            f = fieldgen.iid_field(shape, seed + i)
        out.append(f)
    return out


@pytest.mark.parametrize("dim,n,lo,hi", [(3, 37, 2, 40), (3, 16, 30, 70), (3, 1, 5, 9),
                                         (2, 40, 2, 300)])
def test_batch_matches_oracle(ctx, dev, dim, n, lo, hi):
    """More than one launch group (16 fields each) and a ragged last group;
    sizes from 2 (every vertex on the boundary) upward, odd and even rows."""
    fs = _fields(100 + n + dim, n, dim, lo, hi)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    log("batch", dim, n, "fields, vertices", sum(f.size for f in fs))
    r = pc.classify_batch(ts, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    assert r.status == 0
    assert r.offsets[0] == 0 and np.all(np.diff(r.offsets) >= 0)
    for i, f in enumerate(fs):
        ref = oracle.classify(f)
        got = r.field_list(i).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref.crit), (i, f.shape)
        assert np.array_equal(r.codes[i].cpu().numpy(), ref.codes), (i, f.shape)
        a, b = r.offsets[i], r.offsets[i + 1]
        assert np.array_equal(r.crit_codes[a:b].cpu().numpy(), ref.codes.ravel()[ref.crit])
        d = pc.classify(ts[i], ctx=ctx)
        assert torch.equal(d.codes, r.codes[i]) and torch.equal(d.crit, r.field_list(i))


def test_batch_async_offsets(ctx, dev):
    fs = _fields(7, 20, 3, 10, 33)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    sync = pc.classify_batch(ts, ctx=ctx)
    offs = torch.full((21,), -7, dtype=torch.int64, device=dev)
    asy = pc.classify_batch(ts, ctx=ctx, offsets_dev=offs)
    torch.cuda.synchronize()
    assert asy.offsets is None
    assert np.array_equal(offs.cpu().numpy(), sync.offsets)
    n = int(sync.offsets[-1])
    assert torch.equal(asy.crit[:n], sync.crit[:n])


def test_batch_capacity_and_nan(ctx, dev):
    fs = _fields(9, 5, 3, 8, 20)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    full = pc.classify_batch(ts, ctx=ctx)
    need = int(full.offsets[-1])
    small = pc.classify_batch(ts, ctx=ctx, capacity=need - 1, check=False)
    assert small.status == pc.E_CAPACITY
    assert np.array_equal(small.offsets, full.offsets)
    assert torch.equal(small.crit[:need - 1], full.crit[:need - 1])
    g = fs[3].copy()
    g[1, 2, 3] = np.nan
    ts[3] = torch.from_numpy(g).to(dev)
    assert pc.classify_batch(ts, ctx=ctx, check=False).status == pc.E_NAN


def test_batch_rejects_mixed_dimensions(ctx, dev):
    a = torch.rand(5, 6, 7, device=dev)
    b = torch.rand(6, 7, device=dev)
    with pytest.raises(pc.PcritError) as e:
        pc.classify_batch([a, b], ctx=ctx)
    assert e.value.status == pc.E_ARG


def test_batch_in_captured_graph(ctx, dev):
    """The batch call (device offsets) captured in a graph: replays with eager
    work in between give the eager call's codes, lists and offsets each
    time."""
    fs = _fields(11, 20, 3, 12, 40)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    ref = pc.classify_batch(ts, ctx=ctx)
    n = int(ref.offsets[-1])
    total = sum(f.size for f in fs)
    codes = [torch.zeros(t.shape, dtype=torch.uint8, device=dev) for t in ts]
    crit = torch.empty(total, dtype=torch.int32, device=dev)
    offs = torch.empty(len(ts) + 1, dtype=torch.int64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up: scratch grown before capture
        pc.classify_batch(ts, ctx=ctx, codes=codes, crit=crit, offsets_dev=offs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pc.classify_batch(ts, ctx=ctx, codes=codes, crit=crit, offsets_dev=offs)
    for rep in range(3):
        for c in codes:
            c.zero_()
        crit.fill_(-1)
        offs.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(offs.cpu().numpy(), ref.offsets), rep
        assert torch.equal(crit[:n], ref.crit[:n]), rep
        for c, r in zip(codes, ref.codes):
            assert torch.equal(c, r), rep
