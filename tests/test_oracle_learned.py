"""Pins of the learned-order oracle (``oracle/learned.py``) against facts
that do not come from the oracle itself: finite differences, the integral
definition of the normal distribution, closed forms of linear fields and of
one-point code arrays, direct counts, the closed form of Adam's first step,
and torch's own BF16 conversion."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import learned as L


def test_bf16_round_ties_to_even_and_torch():
    one = 1.0
    u = 2.0 ** -8  # half a BF16 ulp at 1
    vals = np.array([one, one + u, one + 3 * u, one + u + 2.0 ** -20, -one - u,
                     3.0e-39, 65504.0, 1.0e-3], np.float32)
    r = L.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie, even mantissa below
    assert r[2] == one + 4 * u            # tie, even mantissa above
    assert r[3] == one + 2 * u            # above the tie
    assert r[4] == -1.0
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r, ref)
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000)).astype(np.float32)
    assert np.array_equal(L.bf16_round(x),
                          torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy())


def test_gelu_integral_definition():
    pdf = lambda t: math.exp(-0.5 * t * t) / math.sqrt(2.0 * math.pi)
    for x in (-4.0, -1.5, -0.3, 0.0, 0.2, 1.0, 2.5, 6.0):
        cdf = 0.5 + integrate.quad(pdf, 0.0, x, epsabs=1e-14, epsrel=1e-14)[0]
        assert abs(L.gelu(np.array([x]))[0] - x * cdf) < 1e-12
        h = 1e-5
        fd = (L.gelu(np.array([x + h]))[0] - L.gelu(np.array([x - h]))[0]) / (2 * h)
        assert abs(L.gelu_grad(np.array([x]))[0] - fd) < 1e-8


def _random_params(rng, scale=0.5):
    return (rng.standard_normal(L.N_PARAMS) * scale).astype(np.float32)


def test_forward_single_path_network():
    """One nonzero weight per layer: logit = c GELU(b GELU(a x_i)) picks
    input i, layer-1 unit u and layer-2 unit v by their storage offsets."""
    i, u, v = 5, 17, 42
    a, b, c = 1.5, -0.75, 2.0
    p = np.zeros(L.N_PARAMS, np.float32)
    p[L.OFF_W1 + i * L.N_HID + u] = a
    p[L.OFF_W2 + u * L.N_HID + v] = b
    p[L.OFF_W3 + v] = c
    p[L.OFF_B3] = 0.25
    x = np.zeros((3, L.N_IN))
    x[:, i] = [0.5, -1.0, 2.0]
    x[:, 27] = 1.0  # a unit no weight reads
    Phi = lambda t: 0.5 * (1.0 + math.erf(t / math.sqrt(2.0)))
    z, _ = L.forward(p, x, rounding=False)
    for k in range(3):
        h1 = a * x[k, i] * Phi(a * x[k, i])
        h2 = b * h1 * Phi(b * h1)
        assert abs(z[k] - (c * h2 + 0.25)) < 1e-12
    # with the BF16 rounding only h1 moves (weights and x are on the grid)
    zr, cr = L.forward(p, x)
    assert np.all(cr["h1"] == L.bf16_round(cr["h1"]))
    assert np.allclose(zr, z, atol=2 * abs(b * c) * 2.0 ** -8 * 4)


def test_loss_at_zero_logit():
    p = np.zeros(L.N_PARAMS, np.float32)
    x = np.zeros((7, L.N_IN))
    y = np.array([0, 1, 1, 0, 1, 0, 0])
    assert abs(L.loss_sum(p, x, y) - 7 * math.log(2.0)) < 1e-12
    p[L.OFF_B3] = 2.0
    want = 4 * math.log1p(math.exp(2.0)) + 3 * math.log1p(math.exp(-2.0))
    assert abs(L.loss_sum(p, x, y) - want) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_finite_differences(seed):
    """Every parameter block of the analytic gradient against central
    differences of the mean loss (without the BF16 rounding, so the loss is
    smooth)."""
    rng = np.random.default_rng(seed)
    p = _random_params(rng, 0.4).astype(np.float64)
    n = 24
    x = rng.standard_normal((n, L.N_IN))
    y = rng.integers(0, 2, n)
    g = L.backward(p.astype(np.float32), x, y, rounding=False)
    # the oracle reads params as float32: difference on a float32 copy at a
    # step large enough to be exact there
    p32 = p.astype(np.float32)
    blocks = [(L.OFF_W1, L.OFF_B1), (L.OFF_B1, L.OFF_W2), (L.OFF_W2, L.OFF_B2),
              (L.OFF_B2, L.OFF_W3), (L.OFF_W3, L.OFF_B3), (L.OFF_B3, L.N_PARAMS)]
    h = 2.0 ** -10
    for lo, hi in blocks:
        for k in rng.choice(np.arange(lo, hi), size=min(12, hi - lo), replace=False):
            pp, pm = p32.copy(), p32.copy()
            pp[k] += np.float32(h)
            pm[k] -= np.float32(h)
            fd = (L.loss_sum(pp, x, y, rounding=False) - L.loss_sum(pm, x, y, rounding=False)) / (2 * h * n)
            assert abs(fd - g[k]) < 1e-6 + 1e-5 * abs(g[k]), (lo, k, fd, g[k])


def test_linear_field_features():
    """f = x + 2 y + 4 z: interior differences at stride s are
    s (dx + 2 dy + 4 dz), scaled by their largest magnitude 7 s; a clamped
    axis at the grid's edge contributes 0."""
    nz, ny, nx = 9, 11, 13
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = (x + 2 * y + 4 * z).astype(np.float32)
    for level in (0, 1, 2):
        s = 1 << level
        X = L.features(f, level)
        mz, my, mx = (nz - 1) // s + 1, (ny - 1) // s + 1, (nx - 1) // s + 1
        assert X.shape == (mz * my * mx, 32)
        res = math.log2((min(nx, ny, nz) - 1) / s) / 8
        assert np.all(X[:, 27] == L.bf16_round(np.float32(res)))
        assert np.all(X[:, 28:] == 0)
        for (vz, vy, vx) in [(1, 1, 1), (0, 0, 0), (mz - 1, my - 1, mx - 1), (0, my - 1, 1)]:
            row = X[(vz * my + vy) * mx + vx]
            want = []
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        ex = dx if 0 <= vx + dx < mx else 0
                        ey = dy if 0 <= vy + dy < my else 0
                        ez = dz if 0 <= vz + dz < mz else 0
                        want.append(ex + 2 * ey + 4 * ez)
            want = np.array(want, np.float64)
            mag = np.abs(want).max()
            exp = L.bf16_round((want / mag).astype(np.float32))
            assert np.array_equal(row[:27], exp), (level, vz, vy, vx)
    Xc = L.features(np.full((5, 5, 5), 3.0, np.float32), 1)
    assert np.all(Xc[:, :27] == 0)


def test_labels_single_critical_vertex():
    """Codes all regular (0x09, 0x49 on the boundary) but one vertex p: only
    the level vertex v with v - s/2 <= p < v + s/2 on every axis is nonzero,
    ceil(255 / volume of its clipped cell)."""
    shape = (10, 12, 17)
    rng = np.random.default_rng(4)
    for crit_code in (0x00, 0x12, 0x89):
        for _ in range(6):
            codes = np.full(shape, 0x09, np.uint8)
            codes[0] |= 0x40
            codes[:, :, -1] |= 0x40
            p = tuple(int(rng.integers(0, n)) for n in shape)
            codes[p] = crit_code
            for level in (0, 1, 2, 3):
                s = 1 << level
                lab = L.labels(codes, level)
                dims = [(n - 1) // s + 1 for n in shape]
                v = [min((c + s // 2) // s, d - 1) for c, d in zip(p, dims)]
                # a coordinate past the last level vertex's cell belongs to none
                inside = all((c + s // 2) // s <= d - 1 for c, d in zip(p, dims))
                want = np.zeros(dims, np.uint8)
                if inside:
                    vol = 1
                    for vc, n in zip(v, shape):
                        vol *= min(vc * s + s - s // 2, n) - max(vc * s - s // 2, 0)
                    want[tuple(v)] = math.ceil(255 / vol)
                assert np.array_equal(lab, want.ravel()), (crit_code, p, level)


def test_labels_fractions():
    """All critical: 255 everywhere; every other x-column critical: cells of
    an even number of columns hold exactly half (ceil(127.5) = 128)."""
    shape = (9, 8, 16)
    allc = np.zeros(shape, np.uint8)
    for level in (0, 1, 2):
        assert np.all(L.labels(allc, level) == 255)
    half = np.full(shape, 0x09, np.uint8)
    half[..., ::2] = 0x12
    lab = L.labels(half, 2).reshape(3, 2, 4)
    # x cells [4x - 2, 4x + 2) clipped: columns 0..1 for x = 0 (one even)
    assert np.all(lab[..., 1:] == 128) and np.all(lab[..., 0] == 128)
    lab0 = L.labels(half, 0).reshape(shape)
    assert np.array_equal(lab0, np.where(half == 0x12, 255, 0))


def test_region_scores_direct_count():
    """Zero logits: each region scores half its number of level vertices,
    counted from the level's coordinate ranges."""
    shape = (70, 100, 9)
    edge = 32
    for level in (0, 1, 2, 3):
        s = 1 << level
        mz, my, mx = [(n - 1) // s + 1 for n in shape]
        sc = L.region_scores(np.zeros(mz * my * mx), shape, level, edge)
        nry, nrz = -(-shape[1] // edge), -(-shape[0] // edge)
        assert sc.shape == (nry * nrz,)
        for rz in range(nrz):
            for ry in range(nry):
                cy = len(range(-(-ry * edge // s) * s, min((ry + 1) * edge, shape[1]), s))
                cz = len(range(-(-rz * edge // s) * s, min((rz + 1) * edge, shape[0]), s))
                assert sc[rz * nry + ry] == 0.5 * cy * cz * mx
    big = np.full(mz * my * mx, 40.0)
    assert np.allclose(L.region_scores(big, shape, 3, edge).sum(), mz * my * mx)


def test_adam_first_step_closed_form():
    """After one step from zero moments each parameter moves by
    lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-4, 2, 50)
    q, m, v = L.adam_step(p, g, np.zeros(50), np.zeros(50), 1e-3, 1)
    assert np.allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
