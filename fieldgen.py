"""Seeded synthetic scalar fields on regular grids.

This module only draws inputs.  It holds no part of the classification
arithmetic, so both the CPU oracle (``oracle/``) and the GPU path
(``paper_2009_00083_amd``) can be fed from it without sharing any of the
method's code.

The paper measures on public volumes (Jet 512^3, Foot/Random/Turbulence about
17M vertices, Section 5) that are not available here; the workloads below stand
in for them with the same grid sizes and a mix of smooth structure and noise.

Recipe (all configurations):
  * coordinates along an axis of n samples are i/(n-1), i = 0..n-1;
  * isotropic Gaussians a*exp(-|x-c|^2 / (2 sigma^2)) and random-phase
    sinusoids a*sin(2 pi k.x + phi) are summed in float64 and the sum is
    rounded to float32 once, at the end;
  * parameters come from ``numpy.random.default_rng(seed)`` (PCG64) drawn in
    the order: Gaussian centres (K x D), sigmas (K), amplitudes (K), then the
    sinusoid wave vectors, phases and amplitudes, then the noise (N values in
    C order, z slowest, x fastest).

Both kinds of term factor per axis (a Gaussian is a product of 1D Gaussians, a
sinusoid is the imaginary part of a product of complex exponentials), so each
z-plane is one (n_y x K) @ (K x n_x) matrix product.  The product runs on the
CPU in float64 by default; ``device='cuda'`` runs the same float64 products on
the GPU, which is much faster at 512^3 but may round a few samples differently,
so a test always feeds both sides of a comparison from the same array.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CONFIGS", "gaussian_field", "config_field", "tie_field", "iid_field",
    "device_iid_field",
]


def _axis_coords(n: int) -> np.ndarray:
    if n < 2:
        return np.zeros(max(n, 1))
    return np.arange(n, dtype=np.float64) / (n - 1)


def _gauss_factors(coords, centres, sigma):
    # per axis: exp(-(x - c)^2 / (2 sigma^2)), shape (K, n)
    out = []
    for ax, x in enumerate(coords):
        d = x[None, :] - centres[:, ax][:, None]
        out.append(np.exp(-(d * d) / (2.0 * sigma[:, None] ** 2)))
    return out


def _sin_factors(coords, kvec):
    out = []
    for ax, x in enumerate(coords):
        out.append(np.exp(2j * np.pi * kvec[:, ax][:, None] * x[None, :]))
    return out


def _sum_separable(weights, factors, shape, device=None, imag=False):
    """F[z,y,x] (or F[y,x]) = sum_k w_k * prod_axis factor_axis[k, i_axis]."""
    if len(shape) == 2:
        fy, fx = factors
        a = (fy * weights[:, None]).T  # (ny, K)
        if device is not None:
            import torch
            ta = torch.from_numpy(np.ascontiguousarray(a)).to(device)
            tb = torch.from_numpy(np.ascontiguousarray(fx)).to(device)
            r = ta @ tb
            r = (r.imag if imag else r.real) if r.is_complex() else r
            return r.cpu().numpy()
        r = a @ fx
        return r.imag if imag else (r.real if np.iscomplexobj(r) else r)
    fz, fy, fx = factors
    nz, ny, nx = shape
    k = weights.shape[0]
    b = (fy[:, :, None] * fx[:, None, :]).reshape(k, ny * nx)
    a = (fz * weights[:, None]).T  # (nz, K)
    if device is not None:
        import torch
        tb = torch.from_numpy(np.ascontiguousarray(b)).to(device)
        ta = torch.from_numpy(np.ascontiguousarray(a)).to(device)
        r = ta @ tb
        if r.is_complex():
            r = r.imag if imag else r.real
        return r.cpu().numpy().reshape(nz, ny, nx)
    out = np.empty((nz, ny * nx), dtype=np.float64)
    step = max(1, (1 << 24) // max(1, ny * nx))
    for z0 in range(0, nz, step):
        r = a[z0:z0 + step] @ b
        if np.iscomplexobj(r):
            r = r.imag if imag else r.real
        out[z0:z0 + step] = r
    return out.reshape(nz, ny, nx)


def gaussian_field(shape, seed, n_gauss, sigma_range=(0.05, 0.2),
                   amp_range=(-1.0, 1.0), n_sin=0, sin_kmax=16,
                   sin_amp=(0.0, 0.25), noise=None, device=None):
    """Sum of random Gaussians (+ optional sinusoids and noise) as float32.

    ``shape`` is (nz, ny, nx) for 3D or (ny, nx) for 2D (C order, x fastest).
    ``noise`` is None, ('uniform', h) for U[-h, h], or ('normal', s) for
    N(0, s^2).
    """
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_gauss, d))
    sigma = rng.uniform(sigma_range[0], sigma_range[1], size=n_gauss)
    amp = rng.uniform(amp_range[0], amp_range[1], size=n_gauss)
    # centres[:, ax] is the coordinate along array axis ax (z, y, x order)
    coords = [_axis_coords(n) for n in shape]
    f = _sum_separable(amp, _gauss_factors(coords, centres, sigma), shape,
                       device=device)
    if n_sin:
        kv = rng.integers(-sin_kmax, sin_kmax + 1, size=(n_sin, d))
        for i in range(n_sin):
            while not kv[i].any():
                kv[i] = rng.integers(-sin_kmax, sin_kmax + 1, size=d)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=n_sin)
        sa = rng.uniform(sin_amp[0], sin_amp[1], size=n_sin)
        w = sa * np.exp(1j * phi)
        f = f + _sum_separable(w, _sin_factors(coords, kv), shape,
                               device=device, imag=True)
    if noise is not None:
        kind, scale = noise
        n = int(np.prod(shape))
        if kind == "uniform":
            f = f + rng.uniform(-scale, scale, size=n).reshape(shape)
        elif kind == "normal":
            f = f + rng.normal(0.0, scale, size=n).reshape(shape)
        else:
            raise ValueError(kind)
    return np.ascontiguousarray(f.astype(np.float32))


# Workloads (shape in C order).  "direct" = one full-resolution pass,
# "progressive" = coarse-to-fine over every level of the hierarchy.
CONFIGS = {
    # 64^3, 8 Gaussians + U[-1e-3, 1e-3] noise, seed 0
    "gauss64": dict(shape=(64, 64, 64), seed=0, n_gauss=8,
                    noise=("uniform", 1e-3)),
    # 256^3, 64 Gaussians + 32 random-phase sinusoids (|k_i| <= 16), seed 2
    "gsin256": dict(shape=(256, 256, 256), seed=2, n_gauss=64, n_sin=32),
    # 512^3, 256 Gaussians + N(0, 1e-2^2) white noise, seed 3
    "noisy512": dict(shape=(512, 512, 512), seed=3, n_gauss=256,
                     noise=("normal", 1e-2)),
    # 8192^2 2D counterpart of noisy512, seed 4
    "noisy8192": dict(shape=(8192, 8192), seed=4, n_gauss=256,
                      noise=("normal", 1e-2)),
}


def config_field(name, device=None, shape=None):
    """Field of a named workload; ``shape`` overrides the grid size only."""
    kw = dict(CONFIGS[name])
    if shape is not None:
        kw["shape"] = tuple(shape)
    return gaussian_field(device=device, **kw)


def tie_field(shape, seed, levels=3):
    """Integer-valued float32 field with many exact ties (values 0..levels-1)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, levels, size=tuple(shape)).astype(np.float32)


def iid_field(shape, seed):
    """i.i.d. U[0,1) float32 samples."""
    rng = np.random.default_rng(seed)
    return rng.random(size=tuple(shape), dtype=np.float32)


def device_iid_field(shape, seed, device):
    """i.i.d. U[0,1) float32 samples drawn on ``device`` by torch's seeded
    generator there (for grids too large to draw on the host).  Returns a
    device tensor; tests copy the parts the oracle needs from it."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.rand(tuple(shape), generator=g, device=device, dtype=torch.float32)
