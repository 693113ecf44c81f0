"""Pins of the FP64 oracle against mathematics that does not come from it.

Each test targets a mistake that would otherwise go unseen: a wrong weight,
a dropped or doubled centre term, a transposed axis, a wrong sign or index
in the time stepping, the sponge or the adjoint.
"""
from fractions import Fraction
import os

import numpy as np
import pytest

import oracle
from oracle.operators import laplacian, sponge_profile, sponge_field
from synth import COURANT, smooth_random

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_fracs(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line)
    return rows


# ---------------------------------------------------------------- weights

def test_weights_match_textbook_table():
    want = [Fraction(s) for s in _read_fracs("fd_weights_r4.txt")]
    assert oracle.fd_coefficients(4) == want


def test_lower_order_weights_match_textbook_table():
    for row in _read_fracs("fd_weights_low_order.txt"):
        r, rest = row.split(":")
        want = [Fraction(s) for s in rest.split()]
        assert oracle.fd_coefficients(int(r)) == want


def test_symbol_peak_and_stability_bound():
    # peak of |c0 + 2 sum c_m cos(m theta)| at theta = pi, checked on a dense theta grid
    c = oracle.second_derivative_weights(4)
    th = np.linspace(0, np.pi, 20001)
    sym = c[0] + 2 * sum(c[m] * np.cos(m * th) for m in range(1, 5))
    assert np.all(sym <= 1e-15)  # the stencil is a negative operator
    assert abs(np.abs(sym).max() - float(oracle.symbol_peak())) < 1e-12
    assert oracle.symbol_peak() == Fraction(2048, 315)
    # the workloads' time step is half the 3D stability bound
    assert abs(COURANT - 0.5 * oracle.stability_courant()) < 1e-15


# ------------------------------------------------------------- Laplacian

def _grid(shape, h, origin):
    nz, ny, nx = shape
    hx, hy, hz = h
    x = (np.arange(nx) - origin[0]) * hx
    y = (np.arange(ny) - origin[1]) * hy
    z = (np.arange(nz) - origin[2]) * hz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def test_polynomial_exactness_up_to_degree_9():
    """L p == lap p at nodes >= 4 from the boundary, p of degree <= 9 per axis
    (with mixed terms), on an anisotropic grid."""
    shape = (14, 15, 16)
    h = (0.11, 0.13, 0.07)
    X, Y, Z = _grid(shape, h, origin=(8, 7, 7))
    rng = np.random.default_rng(0)
    terms = [(9, 0, 0), (0, 9, 0), (0, 0, 9), (9, 3, 2), (4, 9, 1), (2, 5, 9), (7, 7, 7), (1, 0, 0), (0, 0, 0)]
    p = np.zeros(shape)
    lap = np.zeros(shape)
    for (a, b, cexp) in terms:
        coef = rng.uniform(-1, 1)
        p += coef * X ** a * Y ** b * Z ** cexp
        if a >= 2:
            lap += coef * a * (a - 1) * X ** (a - 2) * Y ** b * Z ** cexp
        if b >= 2:
            lap += coef * b * (b - 1) * X ** a * Y ** (b - 2) * Z ** cexp
        if cexp >= 2:
            lap += coef * cexp * (cexp - 1) * X ** a * Y ** b * Z ** (cexp - 2)
    Lp = laplacian(p, h)
    inner = (slice(4, -4),) * 3
    err = np.abs(Lp[inner] - lap[inner]).max()
    assert err <= 1e-9 * max(1.0, np.abs(lap[inner]).max()), err


def test_degree_10_fails_by_the_exact_constant():
    """For p = x^10 the stencil returns sum_m 2 c_m m^10 h^8 = -1152 h^8 at x = 0
    (exact value 0): the error term of an 8th-order formula."""
    assert sum(2 * c * m ** 10 for m, c in enumerate(oracle.fd_coefficients(4)) if m > 0) == -1152
    for hx in (0.5, 0.25):
        shape = (9, 9, 21)
        X, _, _ = _grid(shape, (hx, 1.0, 1.0), origin=(10, 4, 4))
        Lp = laplacian(X ** 10, (hx, 1.0, 1.0))
        assert abs(Lp[4, 4, 10] - (-1152.0 * hx ** 8)) < 1e-9


@pytest.mark.parametrize("shape,h", [((8, 8, 8), 10.0), ((6, 7, 9), (3.0, 5.0, 7.0))])
def test_dense_brute_force(shape, h):
    A = oracle.dense_laplacian(shape, h)
    rng = np.random.default_rng(1)
    for _ in range(3):
        u = rng.standard_normal(shape)
        got = laplacian(u, h).ravel()
        ref = A @ u.ravel()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    bound = float(oracle.symbol_peak()) * (1 / hx ** 2 + 1 / hy ** 2 + 1 / hz ** 2)
    assert ev.max() < 0
    assert -ev.min() <= bound * (1 + 1e-12)


def test_leapfrog_stability_threshold():
    """Growth sets in exactly where (v dt)^2 lambda_max(-L) crosses 4."""
    shape, h, v = (6, 6, 6), 10.0, 3000.0
    lam = -np.linalg.eigvalsh(oracle.dense_laplacian(shape, h)).min()
    dt_crit = 2.0 / (v * np.sqrt(lam))
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(shape)
    vel = np.full(shape, v)

    def growth(dt):
        out = oracle.forward(vel, h, dt, None, np.zeros(1), np.zeros((0, 3), int), nt=400, init=(u0, u0))
        return np.abs(out["u"]).max() / np.abs(u0).max()

    assert growth(0.98 * dt_crit) < 50
    assert growth(1.02 * dt_crit) > 1e3


# ----------------------------------------------------------- time stepping

def test_energy_conservation_without_source_or_sponge():
    shape, h = (20, 22, 24), 10.0
    vel = smooth_random(shape, seed=7).astype(np.float64)
    dt = COURANT * h / vel.max()
    X, Y, Z = _grid(shape, (h, h, h), origin=(12, 11, 10))
    u0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * 30.0 ** 2))
    state = (u0, u0)
    energies = []
    for _ in range(6):
        out = oracle.forward(vel, h, dt, None, np.zeros(1), np.zeros((0, 3), int), nt=50, init=state)
        # the last step's pair (u^{n+1}, u^n) lives in (u, u_prev)
        energies.append(oracle.discrete_energy(out["u"], out["u_prev"], vel, h, dt))
        state = (out["u"], out["u_prev"])
    e = np.array(energies)
    assert e.min() > 0
    assert np.abs(e - e[0]).max() / e[0] < 1e-11


def test_reciprocity_heterogeneous_velocity():
    """v_s^2 u_{r<-s}(t) = v_r^2 u_{s<-r}(t) for the Dirichlet scheme."""
    shape, h = (18, 17, 16), 10.0
    vel = smooth_random(shape, seed=11).astype(np.float64)
    dt = COURANT * h / vel.max()
    nt = 120
    w = np.random.default_rng(3).standard_normal(nt)
    s, r = (3, 4, 5), (12, 11, 13)
    a = oracle.forward(vel, h, dt, s, w, np.array([r]), nt=nt)["traces"][:, 0]
    b = oracle.forward(vel, h, dt, r, w, np.array([s]), nt=nt)["traces"][:, 0]
    vs2 = vel[s[2], s[1], s[0]] ** 2
    vr2 = vel[r[2], r[1], r[0]] ** 2
    assert np.abs(vs2 * a - vr2 * b).max() <= 1e-11 * np.abs(vs2 * a).max()


def test_source_linearity_and_receivers():
    shape, h = (8, 8, 8), 10.0
    vel = smooth_random(shape, seed=12).astype(np.float64)
    dt = COURANT * h / vel.max()
    rng = np.random.default_rng(4)
    w = rng.standard_normal(30)
    rec = rng.integers(0, 8, size=(10, 3))
    a = oracle.forward(vel, h, dt, (2, 5, 3), w, rec, history=True)
    b = oracle.forward(vel, h, dt, (2, 5, 3), 2 * w, rec)
    assert np.allclose(b["u"], 2 * a["u"], rtol=1e-13, atol=0)
    for n in range(30):  # brute-force receiver sampling
        for k in range(10):
            x, y, z = rec[k]
            assert a["traces"][n, k] == a["history"][n + 1][z, y, x]


def test_first_steps_by_hand():
    """Step 0 puts dt^2 s_0 / dV at the source and nothing else; step 1
    spreads it with exactly the stencil weights times (v dt)^2."""
    shape, h, v = (11, 11, 11), 5.0, 2000.0
    dt = 1e-3
    vel = np.full(shape, v)
    w = np.array([3.0, 0.0])
    out = oracle.forward(vel, h, dt, (5, 5, 5), w, np.zeros((0, 3), int), nt=1)
    q = dt * dt * 3.0 / h ** 3
    expect = np.zeros(shape)
    expect[5, 5, 5] = q
    assert np.array_equal(out["u"], expect)
    out = oracle.forward(vel, h, dt, (5, 5, 5), w, np.zeros((0, 3), int), nt=2)
    c = oracle.second_derivative_weights(4)
    k = (v * dt / h) ** 2
    assert np.isclose(out["u"][5, 5, 5], 2 * q + k * 3 * c[0] * q, rtol=1e-14)
    for m in range(1, 5):
        for pt in ((5, 5, 5 + m), (5, 5 - m, 5), (5 + m, 5, 5)):
            assert np.isclose(out["u"][pt], k * c[m] * q, rtol=1e-14)
    assert out["u"][6, 6, 5] == 0.0  # off-axis: a star stencil, no corners


# ------------------------------------------------------------------ sponge

def test_sponge_profile_values():
    g = sponge_profile(100, 20, 0.015)
    assert g[0] == g[-1] == np.exp(-(0.015 * 20) ** 2)
    assert abs(g[0] - 0.9139311852712282) < 1e-15
    assert g[19] == np.exp(-(0.015) ** 2) and np.all(g[20:80] == 1.0)
    assert np.array_equal(g, g[::-1])
    assert np.all(sponge_profile(30, 0, 0.015) == 1.0)


def test_sponge_literal_equals_one_pass_form():
    """Damping both stored levels equals A^{n+1} = g(2A^n - g A^{n-1} + M L A^n + q)."""
    shape, h = (30, 28, 26), 10.0
    vel = smooth_random(shape, seed=13).astype(np.float64)
    dt = COURANT * h / vel.max()
    W, alpha = 8, 0.05
    w = np.random.default_rng(5).standard_normal(40)
    src = (13, 12, 14)
    lit = oracle.forward(vel, h, dt, src, w, np.zeros((0, 3), int), sponge_width=W, sponge_alpha=alpha)
    g = sponge_field(shape, W, alpha)
    A, Am1 = np.zeros(shape), np.zeros(shape)
    for n in range(40):
        q = np.zeros(shape)
        q[src[2], src[1], src[0]] = dt * dt * w[n] / h ** 3
        A, Am1 = g * (2 * A - g * Am1 + (dt * vel) ** 2 * laplacian(A, h) + q), A
    assert np.abs(A - lit["u"]).max() <= 1e-13 * np.abs(A).max()
    # W = 0 is exactly the Dirichlet run
    d0 = oracle.forward(vel, h, dt, src, w, np.zeros((0, 3), int), sponge_width=0)
    d1 = oracle.forward(vel, h, dt, src, w, np.zeros((0, 3), int), sponge_width=0, sponge_alpha=0.5)
    assert np.array_equal(d0["u"], d1["u"])


# --------------------------------------------------------------- analytic

def _analytic_error(n, h, nt_scale):
    v, f, t0 = 3000.0, 25.0, 1.5 / 25.0
    shape = (n, n, n)
    dt = COURANT * h / v / nt_scale
    T = 0.14  # the pulse has passed; the first boundary reflection arrives later
    nt = int(round(T / dt))
    c = n // 2
    dist = int(round(100.0 / h))
    rec = np.array([[c + dist, c, c], [c, c - dist, c]])
    tt = np.arange(nt) * dt
    w = (1 - 2 * (np.pi * f * (tt - t0)) ** 2) * np.exp(-(np.pi * f * (tt - t0)) ** 2)
    out = oracle.forward(np.full(shape, v), h, dt, (c, c, c), w, rec, nt=nt)
    ref = oracle.point_source_trace((np.arange(nt) + 1) * dt, dist * h, v, f, t0)
    return max(oracle.rel_l2(out["traces"][:, k], ref) for k in range(2))


@pytest.mark.slow
def test_convergence_to_analytic_point_source():
    """Traces approach s(t - r/v) / (4 pi v^2 r) at least at second order
    (2nd-order time, 8th-order space: the observed order lies between) when
    dx and dt are halved together; no boundary reflection reaches the
    receivers inside the window."""
    e1 = _analytic_error(48, 10.0, 1)
    e2 = _analytic_error(96, 5.0, 2)
    order = np.log2(e1 / e2)
    assert e2 < 2e-3, (e1, e2)
    assert order > 1.8, (e1, e2, order)


# ---------------------------------------------------------------- adjoint

def _adjoint_case(seed=21):
    shape, h = (16, 15, 14), 10.0
    vel = smooth_random(shape, seed=seed).astype(np.float64)
    dt = COURANT * h / vel.max()
    nt = 60
    rng = np.random.default_rng(seed)
    rec = np.stack([rng.integers(0, 14, 12), rng.integers(0, 15, 12), rng.integers(0, 16, 12)], axis=1)
    return shape, h, vel, dt, nt, rec, rng


def test_adjoint_dot_product():
    """<F s, d> = <s, F^T d> for F: wavelet -> traces, with the sponge on."""
    shape, h, vel, dt, nt, rec, rng = _adjoint_case()
    W, alpha = 4, 0.08
    src = (7, 6, 8)
    s = rng.standard_normal(nt)
    d = rng.standard_normal((nt, len(rec)))
    Fs = oracle.forward(vel, h, dt, src, s, rec, nt=nt, sponge_width=W, sponge_alpha=alpha)["traces"]
    lam = oracle.adjoint_fields(vel, h, dt, rec, d, sponge_width=W, sponge_alpha=alpha)
    g_src = sponge_field(shape, W, alpha)[src[2], src[1], src[0]]
    Ftd = np.array([dt * dt / h ** 3 * g_src * lam[n + 1][src[2], src[1], src[0]] for n in range(nt)])
    lhs, rhs = float(np.sum(Fs * d)), float(np.dot(s, Ftd))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("W", [0, 4])
def test_gradient_matches_central_differences(W):
    shape, h, vel, dt, nt, rec, rng = _adjoint_case(22)
    alpha = 0.08
    src = (7, 6, 8)
    w = np.sin(np.arange(nt) * 0.3) * np.exp(-((np.arange(nt) - 15) / 6.0) ** 2)
    v_true = vel * (1 + 0.03 * rng.standard_normal(shape))
    d_obs = oracle.forward(v_true, h, dt, src, w, rec, nt=nt, sponge_width=W, sponge_alpha=alpha)["traces"]
    grad, J, _ = oracle.gradient(vel, h, dt, src, w, rec, nt, d_obs=d_obs, sponge_width=W, sponge_alpha=alpha)

    def J_of(vv):
        tr = oracle.forward(vv, h, dt, src, w, rec, nt=nt, sponge_width=W, sponge_alpha=alpha)["traces"]
        return oracle.misfit(tr, d_obs)

    dv = rng.standard_normal(shape) * vel
    eps = 1e-6
    fd = (J_of(vel + eps * dv) - J_of(vel - eps * dv)) / (2 * eps)
    assert abs(fd - float(np.sum(grad * dv))) <= 1e-6 * abs(fd)
    for _ in range(3):  # single voxels
        z, y, x = (int(rng.integers(0, n)) for n in shape)
        e = np.zeros(shape)
        e[z, y, x] = 1e-3 * vel[z, y, x]
        fd = (J_of(vel + e) - J_of(vel - e)) / 2e-3 / vel[z, y, x]
        assert abs(fd - grad[z, y, x]) <= 1e-5 * max(abs(fd), np.abs(grad).max() * 1e-3)


def test_scaled_adjoint_is_forward_run_backwards():
    """mu = M G lambda obeys the forward recurrence backwards in time with
    M R^T r injected inside the damping bracket (the form the GPU uses)."""
    shape, h, vel, dt, nt, rec, rng = _adjoint_case(23)
    W, alpha = 4, 0.08
    d = rng.standard_normal((nt, len(rec)))
    lam = oracle.adjoint_fields(vel, h, dt, rec, d, sponge_width=W, sponge_alpha=alpha)
    G = sponge_field(shape, W, alpha)
    M = (dt * vel) ** 2
    mu1, mu2 = np.zeros(shape), np.zeros(shape)
    for k in range(nt, 0, -1):
        inj = np.zeros(shape)
        np.add.at(inj, (rec[:, 2], rec[:, 1], rec[:, 0]), d[k - 1])
        mu = G * (2 * mu1 - G * mu2 + M * laplacian(mu1, h) + M * inj)
        assert np.abs(mu - M * G * lam[k]).max() <= 1e-12 * max(np.abs(mu).max(), 1e-300)
        mu2, mu1 = mu1, mu


# -------------------------------------------------------- float32 floor

def test_float32_floor_of_the_same_loop():
    shape, h = (32, 32, 32), 10.0
    vel = smooth_random(shape, seed=1)
    dt = COURANT * h / 4500.0
    from synth import ricker
    w = ricker(100, dt, 15.0)
    rec = np.array([[x, 16, 4] for x in range(32)])
    a = oracle.forward(vel, h, dt, (16, 16, 16), w, rec, nt=100)
    b = oracle.forward(vel, h, dt, (16, 16, 16), w, rec, nt=100, dtype=np.float32)
    assert oracle.rel_l2(b["u"], a["u"]) < 1e-5


def test_paper_traffic_is_16_bytes_per_point():
    vals = dict(l.split() for l in _read_fracs("paper_traffic.txt"))
    bpp = float(vals["bytes_per_step"]) / float(vals["grid_points"])
    assert abs(bpp - 16.0) < 0.1  # three float32 reads + one float32 write


def test_pointwise_step_equals_full_loop():
    """step_at (25 explicit taps per node) reproduces one step of the full
    loop at every node of a small grid, sponge and source included."""
    shape, h = (12, 11, 13), 10.0
    vel = smooth_random(shape, seed=31).astype(np.float64)
    dt = COURANT * h / vel.max()
    W, alpha = 3, 0.1
    rng = np.random.default_rng(31)
    w = rng.standard_normal(6)
    src = (6, 5, 4)
    fw = oracle.forward(vel, h, dt, src, w[:5], np.zeros((0, 3), int), nt=5, sponge_width=W,
                        sponge_alpha=alpha, history=True)
    A_n, A_nm1 = fw["history"][5], fw["history"][4]
    nxt = oracle.forward(vel, h, dt, src, w, np.zeros((0, 3), int), nt=6, sponge_width=W, sponge_alpha=alpha)["u"]
    zz, yy, xx = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    got = oracle.step_at(pts, A_n, A_nm1, vel, h, dt, src=src, s_n=w[5], sponge_width=W, sponge_alpha=alpha)
    assert np.abs(got - nxt.ravel()).max() <= 1e-13 * np.abs(nxt).max()


# ------------------------------------------------- 16-bit storage scheme

def test_quantizers_round_to_nearest_even():
    from oracle.storage import quantize
    # half: 10 fraction bits, ulp(1) = 2^-10
    assert quantize(1 + 2.0 ** -11, "f16") == 1.0
    assert quantize(1 + 3 * 2.0 ** -11, "f16") == 1 + 2.0 ** -9
    assert quantize(1 + 2.0 ** -11 + 2.0 ** -20, "f16") == 1 + 2.0 ** -10
    assert quantize(65504.0, "f16") == 65504.0 and quantize(-3.0, "f16") == -3.0
    # bfloat16: 7 fraction bits, ulp(1) = 2^-7
    assert quantize(1 + 2.0 ** -8, "bf16") == 1.0
    assert quantize(1 + 3 * 2.0 ** -8, "bf16") == 1 + 2.0 ** -6
    assert quantize(1 + 2.0 ** -8 + 2.0 ** -16, "bf16") == 1 + 2.0 ** -7
    assert quantize(2.0 ** 100 * (1 + 2.0 ** -8), "bf16") == 2.0 ** 100  # float32 range
    assert quantize(-1.5, "bf16") == -1.5


def test_scale_exponent_keeps_magnitudes_below_2_14():
    from oracle.storage import scale_exponent
    assert scale_exponent(1.0) == 13 and scale_exponent(0.75) == 14 and scale_exponent(0.0) == 0
    rng = np.random.default_rng(5)
    for b in 10.0 ** rng.uniform(-25, 25, 200):  # inside the clamp of the exponent
        e = scale_exponent(b)
        assert 2.0 ** 13 <= b * 2.0 ** e < 2.0 ** 14


def test_one_step_growth_bounds_hold():
    """|M L A| <= gamma max|A| on random fields, so the exponent bounds of the
    velocity form hold: |V+| <= max|V| + gamma max|A|, |A+| <= max|A| + that."""
    from oracle.storage import growth_bound_gamma
    shape, h = (10, 11, 12), (10.0, 9.0, 11.0)
    vel = smooth_random(shape, seed=8).astype(np.float64)
    dt = COURANT * 9.0 / vel.max()
    gamma = growth_bound_gamma(vel.max(), h, dt)
    rng = np.random.default_rng(8)
    worst = 0.0
    for _ in range(20):
        A = rng.standard_normal(shape)
        MLA = (dt * vel) ** 2 * laplacian(A, h)
        worst = max(worst, np.abs(MLA).max() / np.abs(A).max())
    assert worst <= gamma
    # checkerboard (the highest-frequency mode) comes close to the bound
    z, y, x = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    cb = (-1.0) ** (x + y + z)
    inner = (slice(4, -4),) * 3
    ratio = np.abs(((dt * vel.max()) ** 2 * laplacian(cb, h))[inner]).max()
    assert 0.9 * gamma <= ratio <= gamma * (1 + 1e-12)


def test_stored_scheme_without_rounding_is_the_plain_loop():
    from oracle.storage import forward_stored
    shape, h = (14, 13, 15), 10.0
    vel = smooth_random(shape, seed=9)
    dt = COURANT * h / 4500.0
    from synth import ricker
    w = ricker(60, dt, 30.0)
    rec = np.array([[x, 6, 3] for x in range(15)])
    a = forward_stored(vel, h, dt, (7, 6, 7), w, rec, 60, "none", sponge_width=3, sponge_alpha=0.1)
    b = oracle.forward(vel, h, dt, (7, 6, 7), w, rec, nt=60, sponge_width=3, sponge_alpha=0.1)
    assert np.abs(a["u"] - b["u"]).max() <= 1e-13 * np.abs(b["u"]).max()
    assert np.abs(a["traces"] - b["traces"]).max() <= 1e-13 * np.abs(b["traces"]).max()
    g = oracle.sponge_field(shape, 3, 0.1)  # V^n = A^n - g A^{n-1}; the loop stores g A^{n-1}
    assert np.abs(a["v"] - (b["u"] - b["u_prev"])).max() <= 1e-13 * np.abs(b["u"]).max()
    for fmt, tol in (("f16", 1e-3), ("bf16", 1e-2)):
        q = forward_stored(vel, h, dt, (7, 6, 7), w, rec, 60, fmt, sponge_width=3, sponge_alpha=0.1)
        assert 0 < oracle.rel_l2(q["u"], b["u"]) < tol
