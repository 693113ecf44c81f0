"""16-bit wavefield storage with a power-of-two scale per field (FP64 arithmetic).

The paper states no precision (it is inferred float32 from the bytes it
measures, Sec. IV-B); the 16-bit form is an extension.  PARITY UNPINNED: no
published value pins this scheme; it is checked against this emulation and
its error against the plain FP64 loop is reported, not bounded.

The scheme (a reading, stated in full so both sides implement it alone).  The
leapfrog state is kept as the pair

    A^n  and  V^n = A^n - g A^{n-1},

so that one step of ``forward`` reads

    V^{n+1} = g (V^n + M L A^n + q^n),      A^{n+1} = g A^n + V^{n+1}

(algebraically the same update).  Storing V instead of A^{n-1} rounds the
step-to-step change relative to its own size; with (A^n, A^{n-1}) stored, the
change (about 20x smaller than A at these frequencies) is only known through
the difference of two rounded fields and the phase error random-walks.

* each stored field X^k (A or V) is S = Q(2^{e} X^k), decoded as S 2^{-e}, where
  Q rounds to the nearest even IEEE half (f16) or bfloat16 (bf16) value;
* the update is evaluated on the decoded fields; A^{n+1} uses the unrounded
  V^{n+1};
* each new field's exponent is chosen before it is written, from bounds that
  hold at every node, with a_X = max |decoded X^n|:
      |V^{n+1}| <= b_V = a_V + gamma a_A + dt^2 |s_n| / dV,
      |A^{n+1}| <= a_A + b_V,
      gamma = M_max (|k_0| + K),  M_max = (v_max dt)^2,
      k_0 = c_0 sum_a h_a^-2,  K = sum_a sum_{m>=1} 2 |c_m| h_a^-2;
  e = 14 - E with bound < 2^E (every stored magnitude below 2^14 < 65504),
  clamped to [-100, 100], and 0 for a zero bound;
* a trace sample is the decoded stored A^{n+1}.
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


def growth_bound_gamma(vmax, h, dt) -> float:
    """gamma with |M L A| <= gamma max|A| at every node."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    c = second_derivative_weights(4)
    s = 1 / hx ** 2 + 1 / hy ** 2 + 1 / hz ** 2
    k0 = c[0] * s
    K = sum(2 * abs(cm) for cm in c[1:]) * s
    return (vmax * dt) ** 2 * (abs(k0) + K)


def scale_exponent(bound: float) -> int:
    if not bound > 0:
        return 0
    _, E = np.frexp(bound)  # bound = f 2^E, 0.5 <= f < 1, so bound < 2^E
    return int(min(100, max(-100, 14 - int(E))))


def forward_stored(vel, h, dt, src, wavelet, rec, nt, fmt, sponge_width=0, sponge_alpha=0.015,
                   dtype=np.float64):
    """Returns dict(u=decoded A^nt, v=decoded V^nt, traces=[nt, nrec], exps=[(e_A, e_V)...]).
    ``dtype`` sets the arithmetic of the update (float64 by default; float32
    measures how far rounding decisions move with the arithmetic alone)."""
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    v = np.asarray(vel, dtype=np.float64)
    w = np.asarray(wavelet, dtype=np.float64)
    rec = np.asarray(rec, dtype=np.int64).reshape(-1, 3)
    M = ((dt * dt) * v * v).astype(dtype)
    G = (sponge_field(v.shape, sponge_width, sponge_alpha) if sponge_width > 0 else np.ones_like(v)).astype(dtype)
    gamma = growth_bound_gamma(float(v.max()), h, dt)
    vol = hx * hy * hz
    h_t = tuple(dtype(x) for x in (hx, hy, hz))
    A = np.zeros(v.shape, dtype=dtype)
    V = np.zeros(v.shape, dtype=dtype)
    traces = np.zeros((nt, len(rec)))
    exps = []
    for n in range(nt):
        q = np.zeros(v.shape, dtype=dtype)
        qmag = 0.0
        if src is not None:
            ix, iy, iz = src
            q[iz, iy, ix] = dt * dt * w[n] / vol
            qmag = dt * dt * abs(w[n]) / vol
        V_new = G * (V + M * laplacian(A, h_t) + q)
        A_new = G * A + V_new
        aA, aV = float(np.abs(A).max()), float(np.abs(V).max())
        bV = aV + gamma * aA + qmag
        eV, eA = scale_exponent(bV), scale_exponent(aA + bV)
        V = (quantize(V_new.astype(np.float64) * 2.0 ** eV, fmt) * 2.0 ** -eV).astype(dtype)
        A = (quantize(A_new.astype(np.float64) * 2.0 ** eA, fmt) * 2.0 ** -eA).astype(dtype)
        traces[n] = A[rec[:, 2], rec[:, 1], rec[:, 0]]
        exps.append((eA, eV))
    return {"u": A.astype(np.float64), "v": V.astype(np.float64), "traces": traces, "exps": exps}
