"""Discrete energy of the source-free, undamped leapfrog (FP64).

For u^{n+1} - 2u^n + u^{n-1} = dt^2 V L u^n with V = diag(v^2) and L
symmetric, taking the inner product with W (u^{n+1} - u^{n-1}), W = V^{-1},
telescopes to the conserved quantity

    E^{n+1/2} = ||u^{n+1} - u^n||_W^2 / dt^2 - <u^{n+1}, L u^n>,

which is positive below the stability limit.
"""
from __future__ import annotations

import numpy as np

from .operators import laplacian


def discrete_energy(u_next, u_cur, vel, h, dt) -> float:
    v = np.asarray(vel, dtype=np.float64)
    d = np.asarray(u_next, dtype=np.float64) - np.asarray(u_cur, dtype=np.float64)
    kinetic = float(np.sum(d * d / (v * v))) / (dt * dt)
    potential = -float(np.sum(np.asarray(u_next, dtype=np.float64) * laplacian(np.asarray(u_cur, dtype=np.float64), h)))
    return kinetic + potential
