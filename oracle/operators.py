"""Spatial operator, sponge and stability bound (FP64).

* ``laplacian``: Eq. 1 (Sec. II) with per-axis weights c_{a,m} = c_m / h_a^2
  and the centre counted once per axis.  Nodes outside the grid are zero
  (every grid node is an unknown; zero-Dirichlet ghosts).
* ``sponge_profile``: Cerjan-type exponential damping strip of width W.  The
  paper's own boundary is CPML-like (Sec. II, Sec. IV-A); the sponge is the
  absorbing layer of the synthetic workloads.
* ``stability_courant``: largest v dt / h for which the 3D leapfrog with this
  stencil is stable, from the peak of the stencil's Fourier symbol.
"""
from __future__ import annotations

import numpy as np

from .coefficients import fd_coefficients, second_derivative_weights

RADIUS = 4


def laplacian(u: np.ndarray, h) -> np.ndarray:
    """(L u) for u indexed [z, y, x]; ``h`` = (hx, hy, hz) or a scalar."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    c = second_derivative_weights(RADIUS)
    R = RADIUS
    p = np.pad(u, R)  # zero ghost nodes
    nz, ny, nx = u.shape
    core = (slice(R, R + nz), slice(R, R + ny), slice(R, R + nx))
    out = np.zeros_like(u)
    for axis, ha in ((2, hx), (1, hy), (0, hz)):
        acc = c[0] * u
        for m in range(1, R + 1):
            plus = list(core)
            minus = list(core)
            plus[axis] = slice(R + m, R + m + u.shape[axis])
            minus[axis] = slice(R - m, R - m + u.shape[axis])
            acc = acc + c[m] * (p[tuple(plus)] + p[tuple(minus)])
        out = out + acc / (ha * ha)
    return out


def sponge_profile(n: int, width: int, alpha: float) -> np.ndarray:
    """1D damping factors g(i), i = 0..n-1: d = distance to the nearer end,
    g = exp(-(alpha (W - d))^2) for d < W, else 1."""
    i = np.arange(n)
    d = np.minimum(i, n - 1 - i)
    g = np.ones(n, dtype=np.float64)
    inside = d < width
    g[inside] = np.exp(-(alpha * (width - d[inside])) ** 2)
    return g


def sponge_field(shape, width: int, alpha: float) -> np.ndarray:
    """g = g_x g_y g_z on a [z, y, x] grid."""
    nz, ny, nx = shape
    gx = sponge_profile(nx, width, alpha)
    gy = sponge_profile(ny, width, alpha)
    gz = sponge_profile(nz, width, alpha)
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def symbol_peak(radius: int = RADIUS):
    """max over theta of |c_0 + 2 sum_m c_m cos(m theta)|, exact rational,
    attained at theta = pi: -c_0 + 2 sum_m |c_m| (signs alternate)."""
    c = fd_coefficients(radius)
    return abs(c[0] + 2 * sum(cm * (-1) ** m for m, cm in enumerate(c) if m > 0))


def stability_courant(ndim: int = 3, radius: int = RADIUS) -> float:
    """Leapfrog u+ = 2u - u- + (v dt)^2 L u is stable iff (v dt)^2 lambda <= 4
    for every eigenvalue magnitude lambda of -L; on a uniform grid
    lambda_max = ndim * peak / h^2, so v dt / h <= 2 / sqrt(ndim * peak)."""
    return 2.0 / float(np.sqrt(ndim * float(symbol_peak(radius))))
