"""CPU oracle of the learned refinement order (test infrastructure).

Only the tests and the CPU-baseline leg of ``bench.py`` use this module; the
GPU library never imports it.  The paper has no learned part: this is the
plain definition of what the library's network, its training gradient, its
inputs, its targets and the region scores compute (the definitions are
restated in ``include/pcrit.h``), written with numpy in float64.  Where the
library rounds to BF16 (network weights, inputs, the first hidden layer's
activations) this module rounds the same values to BF16 (nearest even)
before using them in float64.

Pins (``tests/test_oracle_learned.py``): the backward pass against central
finite differences of the forward pass; GELU against its integral
definition; closed-form inputs of linear fields; targets of fields with one
known critical point; region scores against a direct sum; the first Adam
step against its closed form.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 32, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_IN * N_HID
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
N_PARAMS = OFF_B3 + 1

_erf = np.vectorize(math.erf, otypes=[np.float64])


def bf16_round(a):
    """float32 values rounded to the nearest BF16 (ties to even), as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits_to_float(bits):
    """BF16 bit patterns (uint16) as float64."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def unpack(params):
    p = np.asarray(params, dtype=np.float32)
    assert p.shape == (N_PARAMS,)
    W1 = p[OFF_W1:OFF_B1].reshape(N_IN, N_HID)
    b1 = p[OFF_B1:OFF_W2].astype(np.float64)
    W2 = p[OFF_W2:OFF_B2].reshape(N_HID, N_HID)
    b2 = p[OFF_B2:OFF_W3].astype(np.float64)
    w3 = p[OFF_W3:OFF_B3]
    b3 = float(p[OFF_B3])
    return W1, b1, W2, b2, w3, b3


def forward(params, x, rounding=True):
    """Logits of inputs x (n x 32, float64 values already on the BF16 grid)
    and the intermediates of the backward pass.  rounding=False drops the
    BF16 rounding (a smooth function, for finite-difference checks)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    W1r, W2r, w3r = rnd(W1), rnd(W2), rnd(w3)
    a1 = x @ W1r + b1
    h1 = rnd(gelu(a1).astype(np.float32)) if rounding else gelu(a1)
    a2 = h1 @ W2r + b2
    h2 = gelu(a2)
    z = h2 @ w3r + b3
    return z, dict(a1=a1, h1=h1, a2=a2, h2=h2, W2r=W2r, w3r=w3r)


def loss_sum(params, x, y, rounding=True):
    """Sum over samples of the binary cross-entropy of the logits against
    targets y in [0, 1] (the library's target bytes / 255)."""
    z, _ = forward(params, x, rounding)
    y = np.asarray(y, dtype=np.float64)
    return float(np.sum(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(params, x, y, rounding=True):
    """Gradient of the mean binary cross-entropy with respect to every
    parameter (the BF16 rounding of weights and of h1 taken as the identity
    in the derivative, as the library's kernels do)."""
    z, c = forward(params, x, rounding)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g = np.zeros(N_PARAMS)
    g[OFF_B3] = dz.sum()
    g[OFF_W3:OFF_B3] = c["h2"].T @ dz
    d2 = dz[:, None] * c["w3r"][None, :] * gelu_grad(c["a2"])
    g[OFF_B2:OFF_W3] = d2.sum(0)
    g[OFF_W2:OFF_B2] = (c["h1"].T @ d2).ravel()
    d1 = (d2 @ c["W2r"].T) * gelu_grad(c["a1"])
    g[OFF_B1:OFF_W2] = d1.sum(0)
    g[OFF_W1:OFF_B1] = (x.T @ d1).ravel()
    return g


def features(f, level):
    """Network inputs (n x 32, float64 on the BF16 grid) of every vertex of
    level `level` of the 3D field f (C order z, y, x)."""
    f = np.asarray(f, dtype=np.float32)
    nz, ny, nx = f.shape
    s = 1 << level
    lv = f[::s, ::s, ::s].astype(np.float64)
    mz, my, mx = lv.shape
    pad = np.pad(lv, 1, mode="edge")
    cols = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = pad[1 + dz:1 + dz + mz, 1 + dy:1 + dy + my, 1 + dx:1 + dx + mx]
                # f(v + s d) - f(v) in float32 arithmetic, as the samples are
                cols.append((nb.astype(np.float32) - lv.astype(np.float32)).astype(np.float64))
    v = np.stack(cols, -1).reshape(-1, 27)
    mag = np.abs(v).max(1)
    inv = np.where(mag > 0, 1.0 / np.where(mag > 0, mag, 1.0), 0.0)
    nmin = min(nx, ny, nz) - 1
    res = math.log2(nmin / s) / 8.0
    x = np.zeros((v.shape[0], N_IN))
    x[:, :27] = bf16_round((v.astype(np.float32) * inv.astype(np.float32)[:, None]).astype(np.float32))
    x[:, 27] = bf16_round(np.float32(res))
    return x


def labels(codes, level):
    """Target bytes of the vertices of level `level`: ceil(255 * fraction of
    critical full-resolution vertices within [v - s/2, v + s/2) along every
    axis, clipped to the grid)."""
    codes = np.asarray(codes, dtype=np.uint8)
    nz, ny, nx = codes.shape
    s = 1 << level
    h = s // 2
    crit = (codes & 0xBF) != 0x09
    mz, my, mx = (nz - 1) // s + 1, (ny - 1) // s + 1, (nx - 1) // s + 1
    out = np.zeros((mz, my, mx), np.uint8)
    for z in range(mz):
        z0, z1 = max(z * s - h, 0), min(z * s + s - h, nz)
        for y in range(my):
            y0, y1 = max(y * s - h, 0), min(y * s + s - h, ny)
            for x in range(mx):
                x0, x1 = max(x * s - h, 0), min(x * s + s - h, nx)
                cell = crit[z0:z1, y0:y1, x0:x1]
                out[z, y, x] = -(-255 * int(cell.sum()) // cell.size)
    return out.ravel()


def region_scores(logits, shape, level, edge):
    """Sum of the sigmoid of the logits of level-`level` vertices per region
    (edge `edge` along y and z, full resolution)."""
    nz, ny, nx = shape
    s = 1 << level
    mz, my, mx = (nz - 1) // s + 1, (ny - 1) // s + 1, (nx - 1) // s + 1
    nry, nrz = -(-ny // edge), -(-nz // edge)
    sig = 1.0 / (1.0 + np.exp(-np.asarray(logits, dtype=np.float64))).reshape(mz, my, mx)
    out = np.zeros(nry * nrz)
    for z in range(mz):
        for y in range(my):
            out[((z * s) // edge) * nry + (y * s) // edge] += sig[z, y].sum()
    return out


def adam_step(params, grad, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma and Ba, Algorithm 1) in float64;
    returns the new (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
