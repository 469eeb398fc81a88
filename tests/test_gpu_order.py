"""GPU parity of the order field (ranks by value, ties by index: a
permutation, compared element by element) and of the extremum lists
against the oracle."""
import sys

import numpy as np
import pytest
import torch

import fieldgen
import oracle
from oracle import order as OO
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


def _special(shape, seed):
    rng = np.random.default_rng(seed)
    vals = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 1.4e-45, -1.4e-45, 3e-40,
                     np.finfo(np.float32).max, -np.finfo(np.float32).max, 0.5], np.float32)
    return vals[rng.integers(0, len(vals), size=shape)]


CASES = [("gauss", (33, 40, 68)), ("tie", (20, 17, 9)), ("iid", (5, 6, 7)), ("special", (9, 10, 11)),
         ("tie", (300, 257)), ("gauss", (2, 2, 2)), ("iid", (64, 64, 64)), ("tie", (1000, 4099))]


@pytest.mark.parametrize("gen,shape", CASES)
def test_order_field_matches_oracle(ctx, dev, gen, shape):
    """Tiles of 4096 keys: sizes below one tile, ragged, and many tiles;
    ties everywhere, signed zeros, infinities, subnormals."""
    f = (fieldgen.gaussian_field(shape, 3, 5, noise=("uniform", 1e-3)) if gen == "gauss" else
         fieldgen.tie_field(shape, 4, 3) if gen == "tie" else
         fieldgen.iid_field(shape, 5) if gen == "iid" else _special(shape, 6))
    log("order field", gen, shape)
    rank, srt = pc.order_field(torch.from_numpy(f).to(dev), ctx=ctx)
    r_ref, s_ref = OO.order_field(f)
    assert np.array_equal(rank.cpu().numpy().view(np.uint32), r_ref)
    assert np.array_equal(srt.cpu().numpy().view(np.uint32), s_ref)


def test_order_field_large(ctx, dev):
    """256^3 samples of the smooth recipe (16.7 M keys, 4096 tiles)."""
    f = fieldgen.config_field("gsin256")
    rank, srt = pc.order_field(torch.from_numpy(f).to(dev), ctx=ctx)
    r_ref, s_ref = OO.order_field(f)
    assert np.array_equal(srt.cpu().numpy().view(np.uint32), s_ref)
    assert np.array_equal(rank.cpu().numpy().view(np.uint32), r_ref)


def test_order_field_nan(ctx, dev):
    f = fieldgen.iid_field((10, 11, 12), 1)
    f[3, 4, 5] = np.nan
    with pytest.raises(pc.PcritError) as e:
        pc.order_field(torch.from_numpy(f).to(dev), ctx=ctx)
    assert e.value.status == pc.E_NAN


@pytest.mark.parametrize("shape", [(20, 33, 70), (9, 8, 64), (300, 257), (64, 128)])
def test_extrema_match_oracle(ctx, dev, shape):
    f = fieldgen.iid_field(shape, sum(shape))
    r = pc.classify(torch.from_numpy(f).to(dev), ctx=ctx)
    mn, mx = pc.extrema(r.codes, ctx=ctx)
    ref_min, ref_max = OO.extrema(oracle.classify(f).codes)
    assert np.array_equal(mn.cpu().numpy().view(np.uint32), ref_min)
    assert np.array_equal(mx.cpu().numpy().view(np.uint32), ref_max)


def test_extrema_capacity(ctx, dev):
    f = fieldgen.iid_field((10, 12, 14), 3)
    r = pc.classify(torch.from_numpy(f).to(dev), ctx=ctx)
    mn, mx = pc.extrema(r.codes, ctx=ctx)
    with pytest.raises(pc.PcritError) as e:
        pc.extrema(r.codes, ctx=ctx, capacity=mn.numel() + mx.numel() - 1)
    assert e.value.status == pc.E_CAPACITY
