"""One leapfrog step evaluated at selected nodes only (FP64).

Used to check outputs of grids too large for the full oracle loop: given the
two stored levels A^n and A^{n-1} (as float arrays of the whole grid), the
one-pass form of the update

    A^{n+1}(p) = g(p) (2 A^n(p) - g(p) A^{n-1}(p) + dt^2 v(p)^2 (L A^n)(p) + q^n(p))

is evaluated at each requested node p by summing the 25 taps of Eq. 1
(Sec. II) explicitly, with zero outside the grid.
"""
from __future__ import annotations

import numpy as np

from .coefficients import second_derivative_weights
from .operators import sponge_profile


def step_at(points, A_n, A_nm1, vel, h, dt, src=None, s_n=0.0, sponge_width=0, sponge_alpha=0.015):
    """points: int array [k, 3] of (ix, iy, iz); arrays indexed [z, y, x]."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    nz, ny, nx = A_n.shape
    c = second_derivative_weights(4)
    gx = sponge_profile(nx, sponge_width, sponge_alpha)
    gy = sponge_profile(ny, sponge_width, sponge_alpha)
    gz = sponge_profile(nz, sponge_width, sponge_alpha)
    out = np.empty(len(points), dtype=np.float64)

    def at(x, y, z):
        if 0 <= x < nx and 0 <= y < ny and 0 <= z < nz:
            return float(A_n[z, y, x])
        return 0.0

    for k, (x, y, z) in enumerate(np.asarray(points, dtype=np.int64)):
        lap = 0.0
        for (dxv, dyv, dzv), ha in (((1, 0, 0), hx), ((0, 1, 0), hy), ((0, 0, 1), hz)):
            acc = c[0] * at(x, y, z)
            for m in range(1, 5):
                acc += c[m] * (at(x + m * dxv, y + m * dyv, z + m * dzv) + at(x - m * dxv, y - m * dyv, z - m * dzv))
            lap += acc / (ha * ha)
        g = gx[x] * gy[y] * gz[z]
        v = float(vel[z, y, x])
        val = 2.0 * float(A_n[z, y, x]) - g * float(A_nm1[z, y, x]) + dt * dt * v * v * lap
        if src is not None and (x, y, z) == tuple(src):
            val += dt * dt * s_n / (hx * hy * hz)
        out[k] = g * val
    return out
