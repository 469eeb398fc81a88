"""Pins of the order-field oracle (``oracle/order.py``) against facts that do
not come from it: pairwise brute force, closed forms, and the
classification oracle (a field and its order field have the same critical
points, since the classification orders vertices the same way)."""
import numpy as np
import pytest

import fieldgen
import oracle
from oracle import order as OO


def _brute_rank(v):
    v = [float(x) for x in np.asarray(v, np.float32).ravel()]
    n = len(v)
    return np.array([sum(1 for j in range(n) if v[j] < v[i] or (v[j] == v[i] and j < i))
                     for i in range(n)], np.uint32)


@pytest.mark.parametrize("seed", range(4))
def test_rank_brute_force(seed):
    rng = np.random.default_rng(seed)
    vals = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 0.5, 3e-40], np.float32)
    v = vals[rng.integers(0, len(vals), 257)] if seed % 2 else \
        rng.standard_normal(300).astype(np.float32)
    rank, srt = OO.order_field(v)
    assert np.array_equal(rank, _brute_rank(v))
    assert np.array_equal(rank[srt], np.arange(v.size))


def test_rank_closed_forms():
    n = 1000
    idx = np.arange(n, dtype=np.float32)
    assert np.array_equal(OO.order_field(idx)[0], np.arange(n))
    assert np.array_equal(OO.order_field(-idx)[0], np.arange(n)[::-1])
    assert np.array_equal(OO.order_field(np.full(n, 2.5, np.float32))[0], np.arange(n))
    z = np.zeros(n, np.float32)
    z[::3] = -0.0
    assert np.array_equal(OO.order_field(z)[0], np.arange(n))  # -0 == +0: index order
    with pytest.raises(ValueError):
        OO.order_field(np.array([1.0, np.nan], np.float32))


@pytest.mark.parametrize("gen", ["tie", "gauss", "iid"])
def test_order_field_has_the_same_critical_points(gen):
    shape = (9, 11, 13)
    f = (fieldgen.tie_field(shape, 3, 3) if gen == "tie" else
         fieldgen.gaussian_field(shape, 4, 5) if gen == "gauss" else fieldgen.iid_field(shape, 5))
    rank, _ = OO.order_field(f)
    a = oracle.classify(f)
    b = oracle.classify(rank.astype(np.float32).reshape(shape))
    assert np.array_equal(a.codes, b.codes)
    assert np.array_equal(a.crit, b.crit)


def test_extrema_closed_forms():
    shape = (6, 7, 8)
    f = np.arange(np.prod(shape), dtype=np.float32).reshape(shape)
    mn, mx = OO.extrema(oracle.classify(f).codes)
    assert mn.tolist() == [0] and mx.tolist() == [f.size - 1]
    codes = np.full(10, 0x09, np.uint8)
    codes[[2, 7]] = 0x08      # no lower component: minima
    codes[[4]] = 0x01         # no upper component: maximum
    codes[[9]] = 0x49         # boundary regular
    mn, mx = OO.extrema(codes)
    assert mn.tolist() == [2, 7] and mx.tolist() == [4]
