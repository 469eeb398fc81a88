"""Progressive calls whose finest level runs beside the coarser levels.

When the caller does not watch the levels (no callback, no level times) and
asks for no re-classification count or list codes, and kernel timing is
off, the finest level's classification runs on the caller's stream
while the coarser levels run on the context's second stream, and its
compaction waits for them.  These cases compare that schedule with the
serial one (kernel timing on, or level times) and with the oracle, through
the C ABI, on grids whose finest levels take the quad tiles and on grids
that do not, and replay the asynchronous call (fork and join inside) from
a captured graph.
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


@pytest.fixture(scope="module")
def ctx(dev):
    return pc.Context(0)


def _run(ctx, ft, serial):
    ctx.set_kernel_timing(True if serial else None)
    try:
        p = pc.progressive(ft, ctx=ctx)
        torch.cuda.synchronize()
    finally:
        ctx.set_kernel_timing(None)
    return p


@pytest.mark.parametrize("shape", [(256, 192, 160), (130, 66, 97), (96, 80, 1), (2200, 2000, 1),
                                   (64, 64, 64)])
def test_beside_matches_serial_and_oracle(ctx, dev, shape):
    f = fieldgen.gaussian_field(shape, 17, 6, noise=("uniform", 1e-3)) if shape[2] > 1 else \
        fieldgen.iid_field(shape[:2], 17)
    ft = torch.from_numpy(f).to(dev)
    log("beside", shape)
    a = _run(ctx, ft, serial=False)
    b = _run(ctx, ft, serial=True)
    c = pc.progressive(ft, ctx=ctx, level_times=True)  # watched levels: serial
    torch.cuda.synchronize()
    n = int(a.offsets[-1])
    for other in (b, c):
        assert np.array_equal(a.offsets, other.offsets)
        assert torch.equal(a.crit[:n], other.crit[:n])
        assert torch.equal(a.codes, other.codes)
    assert np.all(np.diff(c.level_ms) >= 0)
    for i, k in enumerate(a.levels):
        ref = oracle.classify(f, level=k)
        got = a.crit[a.offsets[i]:a.offsets[i + 1]].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref.crit), k
    assert np.array_equal(a.codes.cpu().numpy(), oracle.classify(f).codes)


def test_beside_async_in_captured_graph(ctx, dev):
    f = fieldgen.gaussian_field((256, 128, 96), 23, 6, noise=("uniform", 1e-3))
    ft = torch.from_numpy(f).to(dev)
    ref = pc.progressive(ft, ctx=ctx)
    torch.cuda.synchronize()
    n = int(ref.offsets[-1])
    codes = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
    crit = torch.empty(n + 16, dtype=torch.int32, device=dev)
    offs = torch.empty(len(ref.offsets), dtype=torch.int64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up: scratch grown before capture
        pc.progressive_async(ft, ctx=ctx, codes=codes, crit=crit, offsets=offs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pc.progressive_async(ft, ctx=ctx, codes=codes, crit=crit, offsets=offs)
    other = torch.from_numpy(fieldgen.iid_field((64, 48, 40), 5)).to(dev)
    for rep in range(3):
        pc.progressive(other, ctx=ctx)  # eager work on the same context between replays
        codes.zero_()
        crit.fill_(-1)
        offs.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(offs.cpu().numpy(), ref.offsets), rep
        assert torch.equal(crit[:n], ref.crit[:n]), rep
        assert torch.equal(codes, ref.codes), rep
