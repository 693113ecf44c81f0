"""Pins of the oracle's CPML boundary (FP64) against mathematics that does not
come from it: the textbook first-derivative weights, polynomial exactness,
the plain scheme when the layer has no damping, and absorption measured
against a domain large enough that its own boundaries stay silent.
"""
from fractions import Fraction
import os

import numpy as np
import pytest

import oracle
from oracle.cpml import cpml_profile, d1, first_derivative_coefficients, forward_cpml
from synth import COURANT, ricker

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_first_derivative_weights_match_textbook_table():
    want = [Fraction(l.strip()) for l in open(os.path.join(GOLDEN, "fd_first_derivative_r4.txt"))
            if l.strip() and not l.startswith("#")]
    assert first_derivative_coefficients(4) == want


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_first_derivative_exact_to_degree_8(axis):
    n, h = 30, 0.7
    x = (np.arange(n) - 11.3) * h
    inner = slice(4, n - 4)
    for k in range(10):
        f1 = x ** k
        shape = [1, 1, 1]
        shape[axis] = n
        u = np.broadcast_to(f1.reshape(shape), (n, n, n)).copy()
        got = np.take(d1(u, axis, h), range(4, n - 4), axis=axis)
        exact = np.broadcast_to((k * x ** (k - 1) if k else 0 * x).reshape(shape), (n, n, n))
        exact = np.take(exact, range(4, n - 4), axis=axis)
        if k <= 8:
            err = np.max(np.abs(got - exact)) / max(1.0, np.max(np.abs(exact)))
            assert err < 1e-9, (k, err)
        else:  # degree 9: exactly the truncation term (R!)^2 / (2R+1)! h^8 u^(9) = h^8 9! / 630
            trunc = h ** 8 * 362880 / 630
            assert np.allclose(np.abs(got - exact), trunc, rtol=1e-6), (k, np.max(np.abs(got - exact)), trunc)


def test_profile_is_zero_inside_and_monotone_in_the_layer():
    a, b = cpml_profile(60, 12, 10.0, 1e-3, 3000.0, 15.0)
    assert np.all(a[12:48] == 0.0)
    assert np.all(a[:12] < 0) and np.all(a[48:] < 0)
    assert np.all(np.diff(a[:13]) > 0)  # |a| shrinks toward the interior
    assert np.all((b > 0) & (b < 1))


def _case(n, nt, f0=20.0):
    h, v = 10.0, 2500.0
    dt = COURANT * h / v
    vel = np.full((n, n, n), v)
    c = n // 2
    return vel, h, dt, (c, c, c), ricker(nt, dt, f0)


def test_no_damping_is_the_plain_scheme():
    vel, h, dt, src, wav = _case(24, 40)
    rec = np.array([[x, 12, 5] for x in range(24)])
    plain = oracle.forward(vel, h, dt, src, wav, rec, nt=40)
    # reflection coefficient 1: d0 = 0, so a = 0 and the memory variables stay zero
    got = forward_cpml(vel, h, dt, src, wav, rec, 40, width=6, f0=20.0, reflection=1.0)
    assert all(np.all(p == 0) for p in got["psi"]) and all(np.all(z == 0) for z in got["zeta"])
    assert oracle.rel_l2(got["u"], plain["u"]) < 1e-13
    assert oracle.rel_l2(got["traces"], plain["traces"]) < 1e-13


def test_absorbs_better_than_the_sponge_and_dirichlet():
    """A pulse leaves a 36^3 box (layers of 8 nodes); in the box's interior the
    field must match a 76^3 run whose own faces are too far to be heard yet.
    The CPML must beat a Cerjan sponge of the same width, which beats the bare
    zero-Dirichlet faces."""
    n, big, W, nt = 36, 76, 8, 170
    vel, h, dt, src, wav = _case(n, nt, f0=30.0)
    velb, _, _, srcb, _ = _case(big, nt, f0=30.0)
    off = (big - n) // 2
    crop = (slice(off, off + n),) * 3
    ref = oracle.forward(velb, h, dt, srcb, wav, np.zeros((0, 3), int), nt=nt)["u"][crop]
    inner = (slice(W, n - W),) * 3
    # scale: the direct pulse while it crosses the interior (step 60)
    norm = np.linalg.norm(oracle.forward(velb, h, dt, srcb, wav, np.zeros((0, 3), int), nt=60)["u"][crop][inner])
    assert norm > 0

    def err(u):
        return np.linalg.norm(u[inner] - ref[inner]) / norm

    e_cpml = err(forward_cpml(vel, h, dt, src, wav, np.zeros((0, 3), int), nt, width=W, f0=30.0)["u"])
    # Cerjan strength alpha W = 0.36, as for the workloads' sponge (W = 20, alpha = 0.015 -> 0.3)
    e_sponge = err(oracle.forward(vel, h, dt, src, wav, np.zeros((0, 3), int), nt=nt, sponge_width=W,
                                  sponge_alpha=0.045)["u"])
    e_dir = err(oracle.forward(vel, h, dt, src, wav, np.zeros((0, 3), int), nt=nt)["u"])
    print(f"interior error after the reflections return: CPML {e_cpml:.3e} sponge {e_sponge:.3e} "
          f"Dirichlet {e_dir:.3e}")
    assert e_cpml < 2e-3
    assert e_cpml < 0.05 * e_sponge and e_sponge < e_dir
