"""16-bit wavefield storage with a power-of-two scale per field (FP64 arithmetic).

The paper states no precision (it is inferred float32 from the bytes it
measures, Sec. IV-B); the 16-bit form is an extension.  PARITY UNPINNED: no
published value pins this scheme; it is checked against this emulation and
its error against the plain FP64 loop is reported, not bounded.

The scheme (a reading, stated in full so both sides implement it alone):

* each stored field k is S^k = Q(2^{e_k} A^k), decoded as S^k 2^{-e_k}, where Q
  rounds to the nearest even IEEE half (f16) or bfloat16 (bf16) value;
* the step is the one-pass update of ``forward`` evaluated on the decoded
  fields;
* the exponent of the new field is chosen before it is written, from a bound
  that holds for every node:
      |A^{n+1}| <= beta a_n + a_{n-1} + dt^2 |s_n| / dV,
      beta = max(2, |2 + M_max k_0| + M_max K),  M_max = (v_max dt)^2,
      k_0 = c_0 sum_a h_a^-2,  K = sum_a sum_{m>=1} 2 |c_m| h_a^-2,
  where a_k = max |decoded A^k|; e_{n+1} = 14 - E with bound < 2^E (so every
  stored magnitude stays below 2^14 < 65504), clamped to [-100, 100], and 0 for
  a zero bound;
* a trace sample is the decoded stored value.
"""
from __future__ import annotations

import numpy as np

from .coefficients import second_derivative_weights
from .operators import laplacian, sponge_field


def quantize(x, fmt: str) -> np.ndarray:
    """Round to the nearest even value of the 16-bit format (returned as
    float64); fmt "none" keeps float64 (the unquantized scheme)."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "none":
        return x
    if fmt == "f16":
        return x.astype(np.float16).astype(np.float64)
    if fmt == "bf16":
        u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
        return (u.astype(np.uint32)).view(np.float32).astype(np.float64)
    raise ValueError(fmt)


def growth_bound_beta(vmax, h, dt) -> float:
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    c = second_derivative_weights(4)
    s = 1 / hx ** 2 + 1 / hy ** 2 + 1 / hz ** 2
    k0 = c[0] * s
    K = sum(2 * abs(cm) for cm in c[1:]) * s
    M = (vmax * dt) ** 2
    return max(2.0, abs(2 + M * k0) + M * K)


def scale_exponent(bound: float) -> int:
    if not bound > 0:
        return 0
    _, E = np.frexp(bound)  # bound = f 2^E, 0.5 <= f < 1, so bound < 2^E
    return int(min(100, max(-100, 14 - int(E))))


def forward_stored(vel, h, dt, src, wavelet, rec, nt, fmt, sponge_width=0, sponge_alpha=0.015):
    """Returns dict(u=decoded A^nt, traces=[nt, nrec], exps=[e_1..e_nt])."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    v = np.asarray(vel, dtype=np.float64)
    w = np.asarray(wavelet, dtype=np.float64)
    rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
    M = (dt * dt) * v * v
    G = sponge_field(v.shape, sponge_width, sponge_alpha) if sponge_width > 0 else np.ones_like(v)
    beta = growth_bound_beta(float(v.max()), h, dt)
    vol = hx * hy * hz
    A = np.zeros_like(v)      # decoded A^n
    Am1 = np.zeros_like(v)    # decoded A^{n-1}
    traces = np.zeros((nt, len(rec)))
    exps = []
    for n in range(nt):
        q = np.zeros_like(v)
        qmag = 0.0
        if src is not None:
            ix, iy, iz = src
            q[iz, iy, ix] = dt * dt * w[n] / vol
            qmag = dt * dt * abs(w[n]) / vol
        exact = G * (2 * A - G * Am1 + M * laplacian(A, h) + q)
        e = scale_exponent(beta * np.abs(A).max() + np.abs(Am1).max() + qmag)
        new = quantize(exact * 2.0 ** e, fmt) * 2.0 ** -e
        traces[n] = new[rec[:, 2], rec[:, 1], rec[:, 0]]
        exps.append(e)
        Am1, A = A, new
    return {"u": A, "traces": traces, "exps": exps}
