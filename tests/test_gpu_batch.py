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


# ---------------------------------------------------------------------------
# launch configuration and its autotuner


@pytest.mark.parametrize("dim", [3, 2])
def test_batch_configurations_give_the_same_result(dev, dim):
    """Fields per launch (1 .. 16, a ragged last group) and wave tiles per
    field (64 .. 2^20: deepest tiles down to single-step tiles) change the
    launches, never the result: lists, codes, list codes and offsets equal
    the default configuration's, which equals the oracle's."""
    ctx = pc.Context(0)
    fs = _fields(300 + dim, 23, dim, 3, 60 if dim == 3 else 400)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    assert ctx.batch_config() == (16, 512)
    ref = pc.classify_batch(ts, ctx=ctx, with_crit_codes=True)
    torch.cuda.synchronize()
    for i, f in enumerate(fs):
        assert np.array_equal(ref.field_list(i).cpu().numpy().view(np.uint32), oracle.classify(f).crit)
    n = int(ref.offsets[-1])
    for group, want in ((1, 64), (3, 512), (5, 0), (16, 1 << 20), (7, 100), (0, 8192)):
        ctx.set_batch_config(group, want)
        log("batch config", dim, ctx.batch_config())
        r = pc.classify_batch(ts, ctx=ctx, with_crit_codes=True)
        torch.cuda.synchronize()
        assert r.status == 0 and np.array_equal(r.offsets, ref.offsets), (group, want)
        assert torch.equal(r.crit[:n], ref.crit[:n]) and torch.equal(r.crit_codes[:n], ref.crit_codes[:n])
        for a, b in zip(r.codes, ref.codes):
            assert torch.equal(a, b), (group, want)
    ctx.set_batch_config(0, 0)
    assert ctx.batch_config() == (16, 512)


def test_batch_config_arguments(dev):
    ctx = pc.Context(0)
    for group, want in ((17, 0), (-1, 0), (0, 63), (0, (1 << 20) + 1), (0, -5)):
        with pytest.raises(pc.PcritError) as e:
            ctx.set_batch_config(group, want)
        assert e.value.status == pc.E_ARG
    assert ctx.batch_config() == (16, 512)


def test_batch_autotune(dev):
    """The tuner times every candidate, keeps the fastest in the context, and
    leaves the batch's result in its buffers; later batch calls use the
    choice and give the same result; a batch error comes back unchanged and
    leaves the configuration alone."""
    ctx = pc.Context(0)
    fs = _fields(401, 40, 3, 20, 80)
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    ref = pc.classify_batch(ts, ctx=ctx)
    torch.cuda.synchronize()
    n = int(ref.offsets[-1])
    choice, table, codes, crit, _ = pc.batch_autotune(ts, ctx=ctx, reps=2)
    torch.cuda.synchronize()
    log("autotune", choice, {k: round(v, 3) for k, v in table.items()})
    assert len(table) == pc.binding.BATCH_TUNE_GROUPS.__len__() * len(pc.binding.BATCH_TUNE_WANTS)
    assert all(v > 0 for v in table.values())
    assert choice in table and table[choice] == min(table.values())
    assert ctx.batch_config() == choice
    assert torch.equal(crit[:n], ref.crit[:n])
    for a, b in zip(codes, ref.codes):
        assert torch.equal(a, b)
    r = pc.classify_batch(ts, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(r.offsets, ref.offsets) and torch.equal(r.crit[:n], ref.crit[:n])
    # capacity too small: the checking call fails, the configuration stays
    ctx.set_batch_config(4, 512)
    with pytest.raises(pc.PcritError) as e:
        pc.batch_autotune(ts, ctx=ctx, reps=1, capacity=n - 1)
    assert e.value.status == pc.E_CAPACITY
    assert ctx.batch_config() == (4, 512)
