"""Constant-velocity point-source solution in 3D (FP64).

For u_tt = v^2 lap(u) + s(t) delta(x - x_s) in free space the solution is
the retarded potential u(r, t) = s(t - r/v) / (4 pi v^2 r).  The source time
function is the Ricker wavelet, evaluated here from its formula.
"""
from __future__ import annotations

import numpy as np


def ricker_value(t, f, t0):
    a = (np.pi * f * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def point_source_trace(times, r, v, f, t0):
    """u(r, t) for each t in ``times`` (r > 0, metres; v in m/s)."""
    return ricker_value(np.asarray(times, dtype=np.float64) - r / v, f, t0) / (4.0 * np.pi * v * v * r)
