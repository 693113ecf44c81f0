"""Ricker source time function (input generator)."""
from __future__ import annotations

import numpy as np


def ricker(nt: int, dt: float, f: float, t0: float | None = None) -> np.ndarray:
    """s(t_n) = (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = n dt - t0.

    Evaluated in float64 and returned as float32 (the array both solvers
    consume).  ``t0`` defaults to 1/f.
    """
    if t0 is None:
        t0 = 1.0 / f
    tau = np.arange(nt, dtype=np.float64) * dt - t0
    a = (np.pi * f * tau) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)
