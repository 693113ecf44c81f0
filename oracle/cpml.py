"""CPML absorbing boundary for the leapfrog of ``forward`` (FP64, literal).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's own boundary is a convolutional PML (Sec. II and Sec. IV-A cite
CPML; the paper prints no formulas).  Reading taken: the unsplit CPML of the
second-order acoustic equation obtained from the complex frequency-shifted
coordinate stretch d/dx -> (1/s_x) d/dx with s_x = 1 + d_x / (alpha_x + i w)
(kappa = 1).  Applying the stretch twice,

    (1/s_x) d/dx ((1/s_x) dp/dx) = p_xx + d(psi_x)/dx + zeta_x,
    psi_x  = b_x psi_x  + a_x p_x                    (memory of the first derivative)
    zeta_x = b_x zeta_x + a_x (p_xx + d(psi_x)/dx)   (memory of the second)

with the recursive-convolution coefficients b = exp(-(d + alpha) dt),
a = d (b - 1) / (d + alpha), and the same for y and z.  One time step, at
every node, in this order:

    psi_a^n   = b_a psi_a^{n-1} + a_a D1_a p^n
    zeta_a^n  = b_a zeta_a^{n-1} + a_a (D2_a p^n + D1_a psi_a^n)
    p^{n+1}   = 2 p^n - p^{n-1} + dt^2 v^2 sum_a (D2_a p^n + D1_a psi_a^n + zeta_a^n) + q^n

D2_a is the a-axis part of Eq. 1 (centre weight c_0 / h_a^2 once per axis),
D1_a the 8th-order centred first derivative; nodes outside the grid are zero
(for p, psi and zeta).  Profiles over a layer of W nodes at each end of an
axis: depth xi = max(W - i, i - (n - 1 - W), 0) / W, d = d0 xi^2 with
d0 = -3 v_max ln(R) / (2 W h), alpha = pi f0 (1 - xi).  Inside (xi = 0):
d = 0, so a = 0 and psi, zeta stay zero; there the step is the plain leapfrog
(the D1 psi term still reaches W + R nodes in from the faces).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial, log, pi

import numpy as np

from .coefficients import _solve_exact, second_derivative_weights

RADIUS = 4


def first_derivative_coefficients(radius: int = RADIUS):
    """w_1..w_R (Fractions) with sum_m w_m (u(x+m) - u(x-m)) = u'(x) + O(h^(2R)).

    u(x+m) - u(x-m) = 2 sum_k u^(2k+1)(x) m^(2k+1) / (2k+1)!, so the weights
    solve sum_m 2 w_m m^(2k+1) / (2k+1)! = [k == 0] for k = 0..R-1."""
    a = [[Fraction(2 * m ** (2 * k + 1), factorial(2 * k + 1)) for m in range(1, radius + 1)]
         for k in range(radius)]
    b = [Fraction(1 if k == 0 else 0) for k in range(radius)]
    return _solve_exact(a, b)


def cpml_profile(n: int, width: int, h: float, dt: float, vmax: float, f0: float, reflection: float = 1e-3):
    """(a, b) along one axis of n nodes, float64."""
    i = np.arange(n)
    xi = np.maximum(np.maximum(width - i, i - (n - 1 - width)), 0) / max(width, 1)
    d0 = -3.0 * vmax * log(reflection) / (2.0 * width * h) if width > 0 else 0.0
    d = d0 * xi ** 2
    alpha = pi * f0 * (1.0 - xi)
    b = np.exp(-(d + alpha) * dt)
    a = np.where(d > 0, d * (b - 1.0) / np.where(d + alpha > 0, d + alpha, 1.0), 0.0)
    return a, b


def _shift(u, axis, m):
    """u(node + m along axis), zero outside the grid."""
    out = np.zeros_like(u)
    n = u.shape[axis]
    if abs(m) >= n:
        return out
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if m > 0:
        src[axis], dst[axis] = slice(m, n), slice(0, n - m)
    else:
        src[axis], dst[axis] = slice(0, n + m), slice(-m, n)
    out[tuple(dst)] = u[tuple(src)]
    return out


def d1(u, axis, h):
    w = [float(x) for x in first_derivative_coefficients(RADIUS)]
    acc = np.zeros_like(u)
    for m in range(1, RADIUS + 1):
        acc = acc + w[m - 1] * (_shift(u, axis, m) - _shift(u, axis, -m))
    return acc / h


def d2(u, axis, h):
    c = second_derivative_weights(RADIUS)
    acc = c[0] * u
    for m in range(1, RADIUS + 1):
        acc = acc + c[m] * (_shift(u, axis, m) + _shift(u, axis, -m))
    return acc / (h * h)


def memory_update(p, psi, zeta, a, b, axis, h):
    """One time level of the memory variables of one axis, in the order the
    two applications of the stretch require: psi^n from p^n first, then zeta^n
    from D2 p^n and the derivative of that new psi^n.

    Returns (psi^n, zeta^n, stretched second derivative D2 p^n + D1 psi^n +
    zeta^n).  Works for complex p (harmonic forcing in the tests)."""
    psi_new = b * psi + a * d1(p, axis, h)
    second = d2(p, axis, h)
    dpsi = d1(psi_new, axis, h)
    zeta_new = b * zeta + a * (second + dpsi)
    return psi_new, zeta_new, second + dpsi + zeta_new


def forward_cpml(vel, h, dt, src, wavelet, rec, nt, width, f0, reflection=1e-3, vmax=None, dtype=np.float64,
                 snapshots=()):
    """``nt`` leapfrog steps with CPML layers of ``width`` nodes on all six faces.

    Returns ``u``, ``u_prev``, ``traces`` [nt, nrec], the memory variables
    ``psi`` and ``zeta`` (lists over x, y, z of [z, y, x] arrays) and
    ``snapshots`` {n: A^n} for the requested step indices."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    v = np.asarray(vel).astype(dtype)
    vmax = float(np.max(vel)) if vmax is None else vmax
    wavelet = np.asarray(wavelet).astype(dtype)
    rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
    nz, ny, nx = v.shape
    axes = ((2, hx, nx), (1, hy, ny), (0, hz, nz))  # x, y, z
    ab = []
    for axis, ha, n in axes:
        a, b = cpml_profile(n, width, ha, dt, vmax, f0, reflection)
        shape = [1, 1, 1]
        shape[axis] = n
        ab.append((a.reshape(shape).astype(dtype), b.reshape(shape).astype(dtype)))
    cur = np.zeros(v.shape, dtype=dtype)
    prev = np.zeros(v.shape, dtype=dtype)
    psi = [np.zeros(v.shape, dtype=dtype) for _ in axes]
    zeta = [np.zeros(v.shape, dtype=dtype) for _ in axes]
    traces = np.zeros((nt, len(rec)), dtype=dtype)
    vol = dtype(hx) * dtype(hy) * dtype(hz)
    snaps = {}
    for n in range(nt):
        total = np.zeros(v.shape, dtype=dtype)
        for k, (axis, ha, _) in enumerate(axes):
            a, b = ab[k]
            psi[k], zeta[k], term = memory_update(cur, psi[k], zeta[k], a, b, axis, ha)
            total = total + term
        new = 2 * cur - prev + dt * dt * v * v * total
        if src is not None:
            ix, iy, iz = src
            new[iz, iy, ix] += dt * dt * wavelet[n] / vol
        traces[n] = new[rec[:, 2], rec[:, 1], rec[:, 0]]
        prev, cur = cur, new
        if n + 1 in snapshots:
            snaps[n + 1] = cur.copy()
    return {"u": cur, "u_prev": prev, "traces": traces, "psi": psi, "zeta": zeta, "snapshots": snaps}
