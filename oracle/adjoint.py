"""Exact discrete adjoint of ``forward`` and the velocity gradient (FP64).

The paper has no adjoint; its application (Sec. I, subsurface imaging)
motivates one.  Write the forward loop in its one-pass form (algebraically
identical to the literal two-level damping, checked in the tests):

    A^{n+1} = G (2 A^n + M L A^n - G A^{n-1} + q^n),   n = 0..nt-1,
    A^0 = A^{-1} = 0,  M = diag(dt^2 v^2),  G = diag(g),  q^n = dt^2 s_n e_src / dV,

and the misfit J = 1/2 sum_n || R A^{n+1} - d_obs^n ||^2 with residual
r^n = R A^{n+1} - d_obs^n.  Adding sum_n <lambda^{n+1}, -(A^{n+1} - ...)> and
setting the derivative with respect to each A^k to zero (L symmetric):

    lambda^k = 2 G lambda^{k+1} + L(M G lambda^{k+1}) - G^2 lambda^{k+2} + R^T r^{k-1},
    k = nt..1,  lambda^{nt+1} = lambda^{nt+2} = 0,

    dJ/dM = sum_{n=0}^{nt-1} G lambda^{n+1} * (L A^n),     dJ/dv = 2 dt^2 v * dJ/dM.
"""
from __future__ import annotations

import numpy as np

from .forward import forward
from .operators import laplacian, sponge_field


def misfit(traces, d_obs) -> float:
    r = np.asarray(traces, dtype=np.float64) - np.asarray(d_obs, dtype=np.float64)
    return 0.5 * float(np.sum(r * r))


def adjoint_fields(vel, h, dt, rec, resid, sponge_width=0, sponge_alpha=0.015):
    """Return {k: lambda^k} for k = 1..nt, with resid[n] = r^n (shape [nt, nrec])."""
    v = np.asarray(vel, dtype=np.float64)
    resid = np.asarray(resid, dtype=np.float64)
    nt = resid.shape[0]
    rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
    M = (dt * dt) * v * v
    G = sponge_field(v.shape, sponge_width, sponge_alpha) if sponge_width > 0 else np.ones_like(v)
    lam1 = np.zeros_like(v)  # lambda^{k+1}
    lam2 = np.zeros_like(v)  # lambda^{k+2}
    out = {}
    for k in range(nt, 0, -1):
        inj = np.zeros_like(v)
        np.add.at(inj, (rec[:, 2], rec[:, 1], rec[:, 0]), resid[k - 1])
        lam = 2 * G * lam1 + laplacian(M * G * lam1, h) - G * G * lam2 + inj
        out[k] = lam
        lam2, lam1 = lam1, lam
    return out


def gradient(vel, h, dt, src, wavelet, rec, nt, d_obs=None, resid=None,
             sponge_width=0, sponge_alpha=0.015):
    """Velocity gradient of J.  Give either observed data ``d_obs`` (the
    residual is formed from the forward traces) or the residual directly.
    Returns (grad_v, J, traces)."""
    fw = forward(vel, h, dt, src, wavelet, rec, nt=nt, sponge_width=sponge_width,
                 sponge_alpha=sponge_alpha, history=True)
    traces = fw["traces"]
    if resid is None:
        resid = traces - np.asarray(d_obs, dtype=np.float64)
    J = 0.5 * float(np.sum(np.asarray(resid, dtype=np.float64) ** 2))
    lam = adjoint_fields(vel, h, dt, rec, resid, sponge_width, sponge_alpha)
    v = np.asarray(vel, dtype=np.float64)
    G = sponge_field(v.shape, sponge_width, sponge_alpha) if sponge_width > 0 else np.ones_like(v)
    gM = np.zeros_like(v)
    for n in range(nt):
        A = fw["history"][n]
        if n == 0 and not A.any():
            continue
        gM += G * lam[n + 1] * laplacian(A, h)
    grad_v = 2.0 * dt * dt * v * gM
    return grad_v, J, traces
