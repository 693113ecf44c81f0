"""GPU adjoint and velocity gradient against the FP64 oracle's exact adjoint.

The HIP path runs the adjoint on the scaled field mu = m g lambda with the
same fused kernel as the forward step (residual injected at receivers,
imaging term mu^{k+1} L(A^k) accumulated in the same pass) and recomputes the
forward field from checkpoints; the oracle runs the literal lambda recursion
on the full stored history.  Tolerance on the gradient: rel-L2 <= 1e-4 (float32
accumulation over hundreds of steps of two stencils).
"""
import functools

import numpy as np
import pytest

import oracle
from synth import COURANT, ricker, smooth_random, workload
from synth.velocity import smooth_along_z
from synth.workloads import plane_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_GRAD = 1e-4


def _say(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=None)
def case(rec_kind="box", W=4):
    shape = (30, 34, 40)  # (nz, ny, nx)
    h = 10.0
    vel = smooth_random(shape, seed=61)
    dt = COURANT * h / 4500.0
    nt = 150
    wav = ricker(nt, dt, 20.0)
    src = (20, 17, 6)
    if rec_kind == "box":
        rec = plane_receivers(40, 34, 4)
    else:
        rng = np.random.default_rng(61)
        rec = np.stack([rng.integers(0, 40, 300), rng.integers(0, 34, 300), rng.integers(0, 30, 300)], 1)
        rec = rec.astype(np.int32)
        rec[5] = rec[9]
    v_true = (vel * (1 + 0.05 * np.exp(-((np.arange(30) - 18) / 3.0) ** 2))[:, None, None]).astype(np.float32)
    d_obs = oracle.forward(v_true, h, dt, src, wav, rec, nt=nt, sponge_width=W, sponge_alpha=0.06)["traces"]
    fw = oracle.forward(vel, h, dt, src, wav, rec, nt=nt, sponge_width=W, sponge_alpha=0.06)["traces"]
    resid = (fw - d_obs).astype(np.float32)
    grad_ref, _, _ = oracle.gradient(vel, h, dt, src, wav, rec, nt, resid=resid.astype(np.float64),
                                     sponge_width=W, sponge_alpha=0.06)
    return dict(shape=shape, h=h, vel=vel, dt=dt, nt=nt, wav=wav, src=src, rec=rec, resid=resid,
                grad_ref=grad_ref, d_obs=d_obs, W=W)


@functools.lru_cache(maxsize=None)
def case_wide(rec_kind="box"):
    """150 x 40 x 24 nodes: three x tiles and two y tiles of the adjoint's
    64 x 32 shape (the last x tile ragged), so the forward field's x and y
    halos cross tile edges and the residual plane spans several tiles."""
    shape = (24, 40, 150)  # (nz, ny, nx)
    h = 10.0
    vel = smooth_random(shape, seed=71)
    dt = COURANT * h / 4500.0
    nt = 150
    wav = ricker(nt, dt, 20.0)
    src = (75, 20, 6)
    if rec_kind == "box":
        rec = plane_receivers(150, 40, 4)
    else:
        rng = np.random.default_rng(71)
        rec = np.stack([rng.integers(0, 150, 400), rng.integers(0, 40, 400), rng.integers(0, 24, 400)], 1)
        rec = rec.astype(np.int32)
        rec[7] = rec[30]  # a node with two receivers
        rec[8] = rec[30]  # and three
    v_true = (vel * (1 + 0.05 * np.exp(-((np.arange(24) - 14) / 3.0) ** 2))[:, None, None]).astype(np.float32)
    d_obs = oracle.forward(v_true, h, dt, src, wav, rec, nt=nt, sponge_width=4, sponge_alpha=0.06)["traces"]
    fw = oracle.forward(vel, h, dt, src, wav, rec, nt=nt, sponge_width=4, sponge_alpha=0.06)["traces"]
    resid = (fw - d_obs).astype(np.float32)
    grad_ref, _, _ = oracle.gradient(vel, h, dt, src, wav, rec, nt, resid=resid.astype(np.float64),
                                     sponge_width=4, sponge_alpha=0.06)
    return dict(shape=shape, h=h, vel=vel, dt=dt, nt=nt, wav=wav, src=src, rec=rec, resid=resid,
                grad_ref=grad_ref, d_obs=d_obs, W=4)


def gpu_grad(c, **kw):
    from paper_2404_04441_amd import Solver

    s = Solver(torch.from_numpy(c["vel"]).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"],
               sponge_width=c["W"], sponge_alpha=0.06, adjoint=True, nt_max=c["nt"], **kw)
    g = s.adjoint(c["nt"], torch.from_numpy(c["wav"]).cuda(), torch.from_numpy(c["resid"]).cuda())
    out = g.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("rec_kind,W", [("box", 4), ("list", 4), ("box", 0)])
def test_gradient_matches_oracle_adjoint(rec_kind, W):
    c = case(rec_kind, W)
    _say(f"case: adjoint {c['shape']} nt={c['nt']} receivers={rec_kind} sponge={W}")
    g = gpu_grad(c)
    e = oracle.rel_l2(g, c["grad_ref"])
    _say(f"gradient rel-L2 vs FP64 oracle: {e:.3e}")
    assert np.abs(c["grad_ref"]).max() > 0
    assert e <= TOL_GRAD


@pytest.mark.parametrize("rec_kind", ["box", "list"])
def test_gradient_matches_oracle_adjoint_across_tiles(rec_kind):
    c = case_wide(rec_kind)
    _say(f"case: adjoint {c['shape']} nt={c['nt']} receivers={rec_kind} sponge=4 (3 x 2 adjoint tiles)")
    g = gpu_grad(c)
    e = oracle.rel_l2(g, c["grad_ref"])
    _say(f"gradient rel-L2 vs FP64 oracle: {e:.3e}")
    assert np.abs(c["grad_ref"]).max() > 0
    assert e <= TOL_GRAD


@pytest.mark.parametrize("rec_kind", ["box", "list"])
def test_wide_gradient_invariance(rec_kind):
    """Across tile edges too: any checkpoint interval and tile shape (1, 2 or
    4 rows per wavefront, 64- or 128-node-wide tiles) gives the same bits,
    also with an irregular receiver list whose duplicate nodes are summed in
    a fixed order."""
    c = case_wide(rec_kind)
    base = gpu_grad(c)
    for K in (1, 13, 150):
        _say(f"case: wide {rec_kind} ckpt_interval={K}")
        assert np.array_equal(gpu_grad(c, ckpt_interval=K), base), K
    for v in (1, 3, 8):
        _say(f"case: wide {rec_kind} variant={v}")
        assert np.array_equal(gpu_grad(c, variant=v), base), v


def test_adjoint_dot_product():
    """<F dv, d> = <dv, F^T d> for the linearised map F: dv -> d traces: the
    left side by central differences of <traces(v), d> along a smooth random
    direction (float32 forward runs, eps = 1e-2 relative), the right side
    from wave_adjoint with residual d (random normal).  Tolerance 1e-3: on
    this case the central difference's own truncation is 1.5e-4 (FP64
    oracle: 1.5e-4 at eps = 1e-2, 1.5e-6 at 1e-3) and the oracle's float32
    loop lands at 1.2e-4 (at eps = 1e-3 its rounding reaches 1.9e-3)."""
    from paper_2404_04441_amd import Solver

    c = case_wide("box")
    rng = np.random.default_rng(63)
    d = rng.standard_normal((c["nt"], len(c["rec"]))).astype(np.float32)
    nz, ny, nx = c["shape"]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dv = np.zeros(c["shape"])
    for _ in range(6):
        p, q, r = rng.integers(-3, 4, 3)
        dv += np.cos(2 * np.pi * (p * xx / nx + q * yy / ny + r * zz / nz) + rng.uniform(0, 2 * np.pi))
    v0 = c["vel"].astype(np.float64)
    dv = dv / np.abs(dv).max() * v0
    wav = torch.from_numpy(c["wav"]).cuda()
    d_dev = torch.from_numpy(d).cuda()

    def J(v):
        s = Solver(torch.from_numpy(v.astype(np.float32)).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"],
                   sponge_width=4, sponge_alpha=0.06)
        out = float((s.run(c["nt"], wav).double() * d_dev.double()).sum())
        s.close()
        return out

    eps = 1e-2
    lhs = (J(v0 + eps * dv) - J(v0 - eps * dv)) / (2 * eps)
    s = Solver(torch.from_numpy(c["vel"]).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"], sponge_width=4,
               sponge_alpha=0.06, adjoint=True, nt_max=c["nt"])
    g = s.adjoint(c["nt"], wav, d_dev).cpu().numpy().astype(np.float64)
    s.close()
    rhs = float(np.sum(g * dv))
    rel = abs(lhs - rhs) / abs(rhs)
    _say(f"dot product: <F dv, d> = {lhs:.8e}, <dv, F^T d> = {rhs:.8e}, relative difference {rel:.2e}")
    assert rel <= 1e-3


def test_checkpoint_interval_and_variant_invariance():
    """Recomputation from checkpoints is deterministic: any interval, from
    one segment (store all) to a checkpoint every step, any tile shape and
    either cache policy give the same bits."""
    c = case("box", 4)
    base = gpu_grad(c)
    for K in (1, 7, 12, 150):
        _say(f"case: ckpt_interval={K}")
        assert np.array_equal(gpu_grad(c, ckpt_interval=K), base), K
    for v in (1, 2, 3):
        _say(f"case: variant={v}")
        assert np.array_equal(gpu_grad(c, variant=v), base), v
    _say("case: cache_hint=1 (forward and recomputation with the cached policy)")
    assert np.array_equal(gpu_grad(c, cache_hint=1), base)
    _say("case: tune=False (the fixed rule's forward shape)")
    assert np.array_equal(gpu_grad(c, tune=False), base)


def test_gradient_central_differences_float32():
    """J(v) = <traces(v), d> with d the traces of the starting model: the
    adjoint gradient against central differences of J along a smooth
    direction and at 16 single voxels (float32 forward runs, J summed in
    float64).  d is chosen so J does not cancel: with white-noise d the
    float32 rounding of the traces swamps the differences (the oracle's own
    float32 loop then misses by 11%)."""
    from paper_2404_04441_amd import Solver

    c = case("box", 4)
    rng = np.random.default_rng(62)

    def traces(v):
        s = Solver(torch.from_numpy(v.astype(np.float32)).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"],
                   sponge_width=4, sponge_alpha=0.06)
        tr = s.run(c["nt"], torch.from_numpy(c["wav"]).cuda()).cpu().numpy()
        s.close()
        return tr

    v0 = c["vel"].astype(np.float64)
    d = traces(v0)

    def J(v):
        return float(np.sum(traces(v).astype(np.float64) * d))

    s = Solver(torch.from_numpy(c["vel"]).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"], sponge_width=4,
               sponge_alpha=0.06, adjoint=True, nt_max=c["nt"])
    g = s.adjoint(c["nt"], torch.from_numpy(c["wav"]).cuda(), torch.from_numpy(d).cuda()).cpu().numpy()
    s.close()
    zz = np.arange(c["shape"][0])[:, None, None]
    dv = np.broadcast_to(np.sin(zz / 5.0), c["shape"]) * v0
    eps = 1e-3
    fd = (J(v0 + eps * dv) - J(v0 - eps * dv)) / (2 * eps)
    ad = float(np.sum(g.astype(np.float64) * dv))
    _say(f"directional: fd={fd:.6e} adjoint={ad:.6e} rel={abs(fd - ad) / abs(fd):.2e}")
    assert abs(fd - ad) <= 1e-3 * abs(fd)
    # 16 voxels drawn among the 5% largest |gradient| (where float32 differences resolve)
    flat = np.argsort(np.abs(g).ravel())[-int(0.05 * g.size):]
    picks = rng.choice(flat, 16, replace=False)
    worst = 0.0
    for p in picks:
        z, y, x = np.unravel_index(p, c["shape"])
        e = np.zeros(c["shape"])
        step = 1e-2 * v0[z, y, x]
        e[z, y, x] = step
        fdv = (J(v0 + e) - J(v0 - e)) / (2 * step)
        worst = max(worst, abs(fdv - g[z, y, x]) / abs(g[z, y, x]))
    _say(f"16 voxels: worst relative difference {worst:.3e}")
    assert worst <= 1e-1


def test_autograd_function_matches_direct_adjoint():
    from paper_2404_04441_amd.autograd import Geometry, wave_forward

    c = case("box", 4)
    vel = torch.from_numpy(c["vel"]).cuda().requires_grad_(True)
    wav = torch.from_numpy(c["wav"]).cuda()
    geom = Geometry(h=c["h"], dt=c["dt"], nt=c["nt"], src=c["src"], rec=c["rec"], sponge_width=4,
                    sponge_alpha=0.06)
    d_obs = torch.from_numpy(c["d_obs"].astype(np.float32)).cuda()
    traces = wave_forward(vel, wav, geom)
    loss = 0.5 * ((traces - d_obs) ** 2).sum()
    loss.backward()
    resid = (traces.detach() - d_obs).contiguous()
    from paper_2404_04441_amd import Solver
    s = Solver(torch.from_numpy(c["vel"]).cuda(), c["h"], c["dt"], src=c["src"], rec=c["rec"], sponge_width=4,
               sponge_alpha=0.06, adjoint=True, nt_max=c["nt"])
    g = s.adjoint(c["nt"], wav, resid)
    s.close()
    assert torch.equal(vel.grad, g)
    # the residual is 1e-4 of the traces here, so float32 trace rounding is
    # already 1% of it: the oracle is given the GPU's own residual
    ref, _, _ = oracle.gradient(c["vel"], c["h"], c["dt"], c["src"], c["wav"], c["rec"], c["nt"],
                                resid=resid.cpu().numpy().astype(np.float64), sponge_width=4, sponge_alpha=0.06)
    e = oracle.rel_l2(vel.grad.cpu().numpy(), ref)
    _say(f"autograd gradient vs oracle (same residual): {e:.3e}")
    assert e <= TOL_GRAD


def test_config4_gradient_central_differences():
    """The 256^3 x 800 gradient workload (two-layer true model, smoothed
    start, 256 x 256 receivers, sqrt(T) checkpoints): the adjoint gradient of
    J = 1/2 sum (traces - d_obs)^2 against central differences of J with
    h = 1e-2 v at single voxels, float32 forward runs with J summed in
    float64 on the device.  16 voxels are drawn uniformly from z in [8, 248)
    (rng seed 4); 16 more uniformly from the block the waves cross before
    returning, z in [8, 64), x and y in [64, 192) (seed 5).  Per voxel:
    |fd - g| <= 5% |g| + 1e-3 max|g|, the absolute part covering voxels whose
    effect on the traces is below the float32 rounding of two runs."""
    from paper_2404_04441_amd import Solver

    W = workload("gradient")
    v_true = W.velocity()
    v0 = smooth_along_z(v_true, 8.0)
    dev = torch.device("cuda")
    wav = torch.from_numpy(W.wavelet()).to(dev)
    _say(f"case: {W.name} x {W.nt} steps, gradient and 2 x 32 forward runs")
    st = Solver(torch.from_numpy(v_true).to(dev), W.h, W.dt, src=W.src, rec=W.rec)
    d_obs = st.run(W.nt, wav).double()
    st.close()
    s = Solver(torch.from_numpy(v0).to(dev), W.h, W.dt, src=W.src, rec=W.rec, adjoint=True, nt_max=W.nt)
    tr = s.run(W.nt, wav)
    resid = (tr - d_obs.float()).contiguous()
    g = s.adjoint(W.nt, wav, resid).cpu().numpy().astype(np.float64)
    s.close()
    v0_dev = torch.from_numpy(v0).to(dev)

    def J(vdev):
        f = Solver(vdev, W.h, W.dt, src=W.src, rec=W.rec)
        out = 0.5 * float(((f.run(W.nt, wav).double() - d_obs) ** 2).sum())
        f.close()
        return out

    n = W.shape[0]
    r4 = np.random.default_rng(4)
    r5 = np.random.default_rng(5)
    picks = [(int(r4.integers(8, 248)), int(r4.integers(0, n)), int(r4.integers(0, n))) for _ in range(16)]
    picks += [(int(r5.integers(8, 64)), int(r5.integers(64, 192)), int(r5.integers(64, 192))) for _ in range(16)]
    gmax = np.abs(g).max()
    worst = 0.0
    for k, (z, y, x) in enumerate(picks):
        step = 1e-2 * float(v0[z, y, x])
        vp = v0_dev.clone()
        vp[z, y, x] += step
        vm = v0_dev.clone()
        vm[z, y, x] -= step
        fd = (J(vp) - J(vm)) / (2 * step)
        err = abs(fd - g[z, y, x])
        bound = 0.05 * abs(g[z, y, x]) + 1e-3 * gmax
        worst = max(worst, err / bound)
        _say(f"voxel {k:2d} (z={z:3d}, y={y:3d}, x={x:3d}): adjoint {g[z, y, x]: .4e} fd {fd: .4e} "
             f"|diff| / |g|max {err / gmax:.2e}")
    _say(f"worst |fd - g| / bound = {worst:.3f}")
    assert gmax > 0 and worst <= 1.0
