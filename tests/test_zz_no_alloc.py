"""The allocation-free entry point (pcrit_classify_noalloc) against the
ordinary direct entry point (pcrit_classify), through the C ABI.

Both run the same kernels; the allocation-free call keeps its scratch in a
fixed per-GPU device array that every call reuses, so two calls in a row,
the second on a smaller grid, must each give byte-identical codes and lists.
"""
import sys

import numpy as np
import pytest
import torch

import fieldgen
import paper_2009_00083_amd as pc

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(dev):
    return pc.Context(0)


def _both(ctx, dev, f, level, with_codes):
    ft = torch.from_numpy(f).to(dev)
    m = pc.level_dims(f.shape, level)
    cap = m[0] * m[1] * m[2]
    ref = pc.classify(ft, level, ctx=ctx, with_crit_codes=with_codes)
    codes = torch.full(f.shape, 0xEE, dtype=torch.uint8, device=dev)
    ref_codes = torch.full(f.shape, 0xEE, dtype=torch.uint8, device=dev)
    pc.classify(ft, level, ctx=ctx, codes=ref_codes, with_crit_codes=with_codes)
    crit = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    cc = (torch.zeros(cap, dtype=torch.uint8, device=dev) if with_codes
          else None)
    got = pc.classify_noalloc(ft, level, codes, crit, ctx=ctx, crit_codes=cc)
    torch.cuda.synchronize()
    assert got.status == 0 and ref.status == 0
    assert got.count == ref.count
    assert torch.equal(codes, ref_codes)
    assert torch.equal(got.crit, ref.crit)
    if with_codes:
        assert torch.equal(got.crit_codes, ref.crit_codes)
    return got.count


@pytest.mark.parametrize("with_codes", [False, True])
def test_noalloc_two_calls_second_smaller(ctx, dev, with_codes):
    """3D then a smaller 3D grid, then 2D then a smaller 2D grid; levels 0
    and 1; each against pcrit_classify on the same field."""
    cases = [((70, 130, 200), 0), ((21, 19, 67), 0),
             ((70, 130, 200), 1), ((9, 40, 33), 1),
             ((300, 517), 0), ((45, 70), 0)]
    for shape, level in cases:
        log(f"noalloc case shape={shape} level={level} codes={with_codes}")
        f = fieldgen.iid_field(shape, seed=sum(shape) + level)
        n = _both(ctx, dev, f, level, with_codes)
        assert n > 0


def test_noalloc_full_size_then_small(ctx, dev):
    """The largest bench-size level (512^3) then a tiny one: the scratch left
    by the big call must not leak into the small one."""
    log("noalloc case noisy512 level 0, then (5, 6, 7)")
    f = fieldgen.config_field("noisy512", device="cuda")
    _both(ctx, dev, f, 0, False)
    g = fieldgen.iid_field((5, 6, 7), seed=11)
    _both(ctx, dev, g, 0, True)


def test_noalloc_async_count(ctx, dev):
    log("noalloc case async count")
    f = fieldgen.iid_field((33, 64, 129), seed=5)
    ft = torch.from_numpy(f).to(dev)
    ref = pc.classify(ft, 0, ctx=ctx)
    codes = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
    crit = torch.zeros(f.size, dtype=torch.int32, device=dev)
    cnt = torch.full((1,), -3, dtype=torch.int64, device=dev)
    r = pc.classify_noalloc(ft, 0, codes, crit, ctx=ctx, count_dev=cnt)
    assert r.status == 0
    torch.cuda.synchronize()
    n = int(cnt.item())
    assert n == ref.count
    assert torch.equal(crit[:n], ref.crit)


def test_noalloc_rejects_oversized_level(ctx, dev):
    """A level whose bitmask does not fit the fixed scratch is refused before
    anything is enqueued; its buffers stay untouched."""
    log("noalloc case oversized level (rejected on the host)")
    shape = (300, 1024, 1024)  # 4.9 M bitmask words = 39 MB > 32 MiB
    ft = torch.zeros(shape, dtype=torch.float32, device=dev)
    codes = torch.full(shape, 0x5A, dtype=torch.uint8, device=dev)
    crit = torch.zeros(16, dtype=torch.int32, device=dev)
    r = pc.classify_noalloc(ft, 0, codes, crit, ctx=ctx, check=False)
    assert r.status == pc.E_SCRATCH
    torch.cuda.synchronize()
    assert int((codes != 0x5A).sum().item()) == 0
    # level 1 of the same grid fits
    m = pc.level_dims(shape, 1)
    crit1 = torch.zeros(m[0] * m[1] * m[2], dtype=torch.int32, device=dev)
    r1 = pc.classify_noalloc(ft, 1, codes, crit1, ctx=ctx)
    assert r1.status == 0 and r1.count == 2  # constant field: first and last
    del ft, codes
