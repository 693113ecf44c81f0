"""Seeded synthetic velocity models (m/s), float32, indexed ``[z, y, x]``.

Every model is C-ordered with x fastest, i.e. flat index
``x + nx * (y + ny * z)``, the layout the solver library expects.
These are inputs only; nothing here knows about the wave equation.
"""
from __future__ import annotations

import numpy as np

V_MIN = 1500.0
V_MAX = 4500.0


def _draw_modes(seed: int, nmodes: int, kmax: int):
    rng = np.random.default_rng(seed)
    pqr = rng.integers(-kmax, kmax + 1, size=(nmodes, 3))
    for row in pqr:  # a constant mode carries no structure: replace it by (1,0,0)
        if not row.any():
            row[0] = 1
    amp = rng.uniform(0.0, 1.0, size=nmodes)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    return pqr, amp, phase


def smooth_random(shape, seed: int, origin=(0, 0, 0), full_shape=None,
                  nmodes: int = 32, kmax: int = 4) -> np.ndarray:
    """Smooth random field in [1500, 4500] m/s (sum of periodic cosines).

    ``shape`` and ``full_shape`` are ``(nz, ny, nx)``.  The field is defined
    pointwise on the ``full_shape`` grid, so a crop evaluated with
    ``origin=(z0, y0, x0)`` equals the same window of the full field.
    f = sum_k a_k cos(2 pi (p_k x/NX + q_k y/NY + r_k z/NZ) + phi_k),
    v = 3000 + 1500 f / sum_k a_k.
    """
    nz, ny, nx = shape
    NZ, NY, NX = full_shape if full_shape is not None else shape
    z0, y0, x0 = origin
    pqr, amp, phase = _draw_modes(seed, nmodes, kmax)
    xs = (x0 + np.arange(nx)) / NX
    ys = (y0 + np.arange(ny)) / NY
    zs = (z0 + np.arange(nz)) / NZ
    f = np.zeros(shape, dtype=np.float64)
    for (p, q, r), a, ph in zip(pqr, amp, phase):
        ex = np.exp(2j * np.pi * p * xs)
        ey = np.exp(2j * np.pi * q * ys)
        ez = np.exp(2j * np.pi * r * zs) * np.exp(1j * ph)
        f += a * (ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).real
    v = 3000.0 + 1500.0 * f / amp.sum()
    return np.clip(v, V_MIN, V_MAX).astype(np.float32)


def smooth_random_torch(shape, seed: int, device, nmodes: int = 32, kmax: int = 4):
    """The field of :func:`smooth_random` on the full grid, evaluated with
    torch on ``device``: 1D tables in float64, the 3D products in float32, so
    it agrees with the host version to float32 rounding.  Used for grids too
    large to build on the host quickly (1024^3)."""
    import torch

    nz, ny, nx = shape
    pqr, amp, phase = _draw_modes(seed, nmodes, kmax)
    f = torch.zeros(shape, dtype=torch.float32, device=device)
    xs = torch.arange(nx, dtype=torch.float64, device=device) / nx
    ys = torch.arange(ny, dtype=torch.float64, device=device) / ny
    zs = torch.arange(nz, dtype=torch.float64, device=device) / nz
    for (p, q, r), a, ph in zip(pqr, amp, phase):
        # cos(X + Y + Z + ph) expanded so that only 1D tables are float64
        X = 2 * np.pi * p * xs
        Y = 2 * np.pi * q * ys
        Z = 2 * np.pi * r * zs + ph
        cx, sx = torch.cos(X).float(), torch.sin(X).float()
        cy, sy = torch.cos(Y).float(), torch.sin(Y).float()
        cz, sz = torch.cos(Z).float(), torch.sin(Z).float()
        cyx = cy[:, None] * cx[None, :] - sy[:, None] * sx[None, :]
        syx = sy[:, None] * cx[None, :] + cy[:, None] * sx[None, :]
        f.add_(float(a) * (cz[:, None, None] * cyx[None] - sz[:, None, None] * syx[None]))
    v = 3000.0 + 1500.0 * f / float(amp.sum())
    return v.clamp_(V_MIN, V_MAX)


def _interfaces(rng, nz: int, count: int, lo: int, hi: int, min_gap: int):
    for _ in range(10000):
        d = np.sort(rng.integers(lo, hi, size=count))
        if count < 2 or np.diff(d).min() >= min_gap:
            return d
    raise RuntimeError("could not place interfaces")


def _gaussian_smooth(a: np.ndarray, sigma: float, axes) -> np.ndarray:
    from scipy.ndimage import gaussian_filter1d

    for ax in axes:
        a = gaussian_filter1d(a, sigma, axis=ax, mode="wrap", truncate=3.0)
    return a


def layered_perturbed(shape, seed: int, rel_perturbation: float = 0.05,
                      sigma_cells: float = 4.0) -> np.ndarray:
    """Six flat layers (1500..4500 m/s, five random interface depths) times a
    (1 + 5%) Gaussian-smoothed white-noise perturbation of unit RMS."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    lo = max(1, int(round(40 * nz / 512)))
    hi = max(lo + 5, int(round(472 * nz / 512)))
    gap = max(1, int(round(16 * nz / 512)))
    depths = _interfaces(rng, nz, 5, lo, hi, gap)
    layer_v = np.array([1500.0, 2100.0, 2700.0, 3300.0, 3900.0, 4500.0], dtype=np.float32)
    zi = np.searchsorted(depths, np.arange(nz), side="right")
    v_layer = layer_v[zi]  # per z
    p = rng.standard_normal(size=shape, dtype=np.float32)
    p = _gaussian_smooth(p, sigma_cells, axes=(0, 1, 2))
    p /= np.float32(np.sqrt(np.mean(p.astype(np.float64) ** 2)))
    v = v_layer[:, None, None] * (np.float32(1.0) + np.float32(rel_perturbation) * p)
    return np.clip(v, V_MIN, V_MAX).astype(np.float32)


def two_layer(shape, interface: int, v_top: float = 2000.0, v_bottom: float = 3000.0) -> np.ndarray:
    """Two flat layers: ``v_top`` for z < interface, ``v_bottom`` below."""
    nz, ny, nx = shape
    v = np.where(np.arange(nz) < interface, v_top, v_bottom).astype(np.float32)
    return np.broadcast_to(v[:, None, None], shape).copy()


def smooth_along_z(v: np.ndarray, sigma_cells: float) -> np.ndarray:
    """Gaussian smoothing along z only (edges replicated): a starting model."""
    from scipy.ndimage import gaussian_filter1d

    return gaussian_filter1d(v.astype(np.float64), sigma_cells, axis=0, mode="nearest").astype(np.float32)


def layered_profile(nz: int, seed: int) -> np.ndarray:
    """z profile of a serving request's model: 2..6 flat layers at random
    sorted depths with sorted velocities drawn from U[1500, 4500] m/s."""
    rng = np.random.default_rng(seed)
    nlayers = int(rng.integers(2, 7))
    depths = np.sort(rng.choice(np.arange(1, nz), size=nlayers - 1, replace=False))
    vels = np.sort(rng.uniform(V_MIN, V_MAX, size=nlayers))
    zi = np.searchsorted(depths, np.arange(nz), side="right")
    return vels[zi].astype(np.float32)


def request_layered(shape, seed: int) -> np.ndarray:
    """The full 3D model of :func:`layered_profile`."""
    nz, ny, nx = shape
    v = layered_profile(nz, seed)
    return np.broadcast_to(v[:, None, None], shape).copy()
