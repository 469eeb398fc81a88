"""The compaction (bitmask words -> ascending critical list) over many
launches of different chunk counts on one context, through the C ABI.

The context reuses its scratch (bitmask words, per-chunk counts) from launch
to launch: the cases run launches growing, shrinking and repeated in a row
on one fresh context, each list against the oracle and against the
allocation-free entry point (a fixed scratch array of its own), and a direct
call replayed from a captured graph with launches of other sizes on the same
context in between.
"""
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


# chunk counts of the direct level-0 launch: 64-bit words of the rows, in
# chunks of 1024 words (256 for launches of few words)
SHAPES = [(512, 256, 64), (64, 64, 64), (512, 512, 64), (9, 7, 5), (512, 256, 64),
          (130, 70, 33), (512, 512, 64), (2, 2, 2)]


def _field(shape, seed):
    if seed % 2:
        return fieldgen.iid_field(shape, seed)
    return fieldgen.gaussian_field(shape, seed, 6, noise=("uniform", 1e-3))


def test_launch_sequence_matches_oracle(dev):
    """A fresh context, launches of hundreds of chunks down to one and back,
    each list against the oracle and against the allocation-free call."""
    ctx = pc.Context(0)
    refs = {}
    for i, shape in enumerate(SHAPES):
        f = _field(shape, 40 + i % 4)
        key = (shape, 40 + i % 4)
        if key not in refs:
            refs[key] = oracle.classify(f)
        ref = refs[key]
        ft = torch.from_numpy(f).to(dev)
        log("direct", shape)
        r = pc.classify(ft, ctx=ctx)
        torch.cuda.synchronize()
        assert r.status == 0 and r.count == ref.count, shape
        assert np.array_equal(r.crit.cpu().numpy().view(np.uint32), ref.crit), shape
        if f.size <= 512 * 512 * 64:
            codes = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
            crit = torch.full((f.size,), -7, dtype=torch.int32, device=dev)
            g = pc.classify_noalloc(ft, 0, codes, crit, ctx=ctx)
            torch.cuda.synchronize()
            assert g.status == 0 and g.count == r.count
            assert torch.equal(g.crit, r.crit)


def test_repeated_and_async(dev):
    """The same launch many times, the asynchronous count, and the
    progressive driver's one-level launches."""
    ctx = pc.Context(0)
    f = _field((512, 512, 64), 7)
    ref = oracle.classify(f)
    ft = torch.from_numpy(f).to(dev)
    cnt = torch.full((1,), -3, dtype=torch.int64, device=dev)
    for rep in range(12):
        r = pc.classify(ft, ctx=ctx, count_dev=cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == ref.count, rep
        assert np.array_equal(r.crit[:ref.count].cpu().numpy().view(np.uint32), ref.crit), rep
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(p.level_list(0).cpu().numpy().view(np.uint32), ref.crit)
    ref1 = oracle.classify(f, level=1)
    assert np.array_equal(p.level_list(1).cpu().numpy().view(np.uint32), ref1.crit)


def test_in_captured_graph(dev):
    """The direct call with a device count captured in a graph: replays with
    launches of other sizes on the same context in between give the eager
    call's list and count each time."""
    ctx = pc.Context(0)
    f = _field((512, 256, 64), 3)
    ft = torch.from_numpy(f).to(dev)
    ref = pc.classify(ft, ctx=ctx)
    other = torch.from_numpy(_field((512, 512, 64), 5)).to(dev)
    small = torch.from_numpy(_field((40, 30, 20), 6)).to(dev)
    codes = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
    crit = torch.empty(f.size, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up: scratch grown before capture
        pc.classify(other, ctx=ctx)
        pc.classify(ft, ctx=ctx, codes=codes, crit=crit, count_dev=cnt, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pc.classify(ft, ctx=ctx, codes=codes, crit=crit, count_dev=cnt)
    for rep in range(4):
        # other launches on the same context overwrite its scratch
        pc.classify(other if rep % 2 else small, ctx=ctx)
        crit.fill_(-1)
        cnt.fill_(-9)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(cnt.item()) == ref.count, rep
        assert torch.equal(crit[:ref.count], ref.crit), rep
        assert torch.equal(codes, ref.codes), rep


@pytest.mark.parametrize("kind", ["checker", "checker_rows", "half"])
def test_dense_rounds(dev, kind):
    """Rounds of 64 words with most bits set (checkerboards: most vertices
    critical) and mixed ones: lists and list codes against the oracle, on
    full-resolution levels (linear words) and on level 1 (row starts from
    the word's row)."""
    ctx = pc.Context(0)
    shape = (256, 96, 40)
    x, y, z = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    f = ((-1.0) ** (x + y + z)).astype(np.float32) + 1e-3 * fieldgen.iid_field(shape, 3)
    if kind == "checker_rows":
        f = np.where(y % 3 == 0, fieldgen.iid_field(shape, 4), f).astype(np.float32)
    elif kind == "half":
        f = np.where(fieldgen.iid_field(shape, 5) < 0.5, f, fieldgen.iid_field(shape, 6))
        f = f.astype(np.float32)
    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    for level in (0, 1):
        ref = oracle.classify(f, level=level)
        log(kind, "level", level, "critical fraction", ref.count / ref.codes.size * (8 if level else 1))
        r = pc.classify(ft, level, ctx=ctx, with_crit_codes=True)
        torch.cuda.synchronize()
        assert r.count == ref.count
        assert np.array_equal(r.crit.cpu().numpy().view(np.uint32), ref.crit)
        assert np.array_equal(r.crit_codes.cpu().numpy(), ref.codes.ravel()[ref.crit])
    p = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(p.level_list(0).cpu().numpy().view(np.uint32), oracle.classify(f).crit)
