"""Finite-difference weights c_0..c_R of Eq. 1 (Sec. II), as exact rationals.

Eq. 1 approximates each second derivative by a symmetric sum over
m = 0..R of c_m [u(+m) + u(-m)].  The paper calls the c's "discretization
parameters" and does not print them; the order (8th in space, R = 4) is
stated in Sec. II and Sec. IV-A.  Here they are derived from the Taylor
expansion: u(x+mh) + u(x-mh) = 2 sum_k u^(2k)(x) (mh)^(2k)/(2k)!, so the
stencil equals h^2 u'' + O(h^(2R+2)) iff

    sum_{m=1..R} 2 c_m m^(2k) / (2k)! = [k == 1]     for k = 1..R,
    c_0 = -2 sum_{m>=1} c_m                            (k = 0).

Solved with fraction-exact Gaussian elimination.  c_0 is the full centre
weight of one axis (the reading of Eq. 1's doubled m = 0 term).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial


def _solve_exact(a, b):
    n = len(b)
    m = [list(row) + [rhs] for row, rhs in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col] / m[col][col]
                m[r] = [x - f * y for x, y in zip(m[r], m[col])]
    return [m[i][n] / m[i][i] for i in range(n)]


def fd_coefficients(radius: int = 4):
    """Return [c_0, c_1, ..., c_R] as Fractions (unit grid spacing)."""
    a = [[Fraction(2 * m ** (2 * k), factorial(2 * k)) for m in range(1, radius + 1)]
         for k in range(1, radius + 1)]
    b = [Fraction(1 if k == 1 else 0) for k in range(1, radius + 1)]
    c = _solve_exact(a, b)
    c0 = -2 * sum(c)
    return [c0] + c


def second_derivative_weights(radius: int = 4):
    """The same weights as floats."""
    return [float(c) for c in fd_coefficients(radius)]
