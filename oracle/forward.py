"""Forward time stepping, written out literally (FP64).

Sec. II: Eq. 1 is evaluated at every grid point in each time step to advance
the wavefield.  The paper does not name the integrator;
the reading taken is the 2nd-order leapfrog of the constant-density acoustic
equation u_tt = v^2 lap(u) + s(t) delta(x - x_s):

    new = 2 cur - prev + dt^2 v^2 L(cur)
    new[src] += dt^2 s(t_n) / (dx dy dz)          (discrete point source)
    new <- g new ;  cur <- g cur                    (Cerjan: damp both levels)
    trace[n, r] = new[rec_r]                        (nodal receivers)
    prev, cur <- cur, new

starting from prev = cur = 0 unless an initial state is given.
"""
from __future__ import annotations

import numpy as np

from .operators import laplacian, sponge_field


def forward(vel, h, dt, src, wavelet, rec, nt=None, sponge_width=0, sponge_alpha=0.015,
            init=None, history=False, dtype=np.float64):
    """Run ``nt`` steps.

    vel      : [z, y, x] velocity (m/s)
    h        : scalar or (hx, hy, hz)
    src      : (ix, iy, iz) or None
    wavelet  : s(t_n), n = 0..nt-1 (ignored when src is None)
    rec      : int array [nrec, 3] of (ix, iy, iz)
    init     : optional (u^0, stored previous level) pair
    history  : also return [A^0, A^1, ..., A^nt]

    Returns a dict with ``u`` (the field after the last step), ``u_prev`` (the
    stored previous level, damped), ``traces`` [nt, nrec] and optionally
    ``history``.  ``dtype`` may be set to float32 to measure the float32
    rounding floor of the same loop.
    """
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    v = np.asarray(vel).astype(dtype)
    wavelet = np.asarray(wavelet).astype(dtype)
    if nt is None:
        nt = len(wavelet)
    rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
    if init is None:
        cur = np.zeros(v.shape, dtype=dtype)
        prev = np.zeros(v.shape, dtype=dtype)
    else:
        cur = np.asarray(init[0]).astype(dtype).copy()
        prev = np.asarray(init[1]).astype(dtype).copy()
    g = sponge_field(v.shape, sponge_width, sponge_alpha).astype(dtype) if sponge_width > 0 else None
    dt = dtype(dt)
    vol = dtype(hx) * dtype(hy) * dtype(hz)
    traces = np.zeros((nt, len(rec)), dtype=dtype)
    hist = [cur.copy()] if history else None
    h_typed = tuple(dtype(a) for a in (hx, hy, hz))
    for n in range(nt):
        lap = laplacian(cur, h_typed)
        new = 2 * cur - prev + dt * dt * v * v * lap
        if src is not None:
            ix, iy, iz = src
            new[iz, iy, ix] += dt * dt * wavelet[n] / vol
        if g is not None:
            new = g * new
            cur = g * cur
        traces[n] = new[rec[:, 2], rec[:, 1], rec[:, 0]]
        prev, cur = cur, new
        if history:
            hist.append(cur.copy())
    out = {"u": cur, "u_prev": prev, "traces": traces}
    if history:
        out["history"] = hist
    return out
