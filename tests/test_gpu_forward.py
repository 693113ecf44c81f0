"""GPU parity of the fused forward step against the FP64 oracle (through the C ABI).

Tolerance: relative L2 <= 1e-5 on the final field for float32 storage (the
target the solver is specified to), accumulated in float64.
"""
import functools

import numpy as np
import pytest

import oracle
from synth import COURANT, ricker, smooth_random, workload
from synth.workloads import line_receivers, plane_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_F32 = 1e-5


def _say(*a):
    print(*a, flush=True)


def gpu_run(vel, h, dt, src, wavelet, rec, nt, **kw):
    from paper_2404_04441_amd import Solver

    v = torch.from_numpy(np.ascontiguousarray(vel, dtype=np.float32)).cuda()
    s = Solver(v, h, dt, src=src, rec=rec, **kw)
    w = torch.from_numpy(np.ascontiguousarray(wavelet, dtype=np.float32)).cuda() if src is not None else None
    tr = s.run(nt, w)
    u, up = s.read_field(0), s.read_field(1)
    torch.cuda.synchronize()
    out = dict(u=u.cpu().numpy(), u_prev=up.cpu().numpy(), traces=None if tr is None else tr.cpu().numpy())
    s.close()
    return out


@functools.lru_cache(maxsize=None)
def small_case():
    W = workload("small")
    vel = W.velocity()
    wav = W.wavelet()
    ref = oracle.forward(vel, W.h, W.dt, W.src, wav, W.rec, nt=W.nt)
    return W, vel, wav, ref


def test_small_workload_parity():
    W, vel, wav, ref = small_case()
    _say("case: small 64^3, 200 steps, f32")
    got = gpu_run(vel, W.h, W.dt, W.src, wav, W.rec, W.nt)
    e_u = oracle.rel_l2(got["u"], ref["u"])
    e_tr = oracle.rel_l2(got["traces"], ref["traces"])
    # the stored previous level is undamped (no sponge here: equal to the oracle's)
    e_up = oracle.rel_l2(got["u_prev"], ref["u_prev"])
    _say(f"rel-L2 u={e_u:.3e} u_prev={e_up:.3e} traces={e_tr:.3e}")
    assert e_u <= TOL_F32 and e_up <= TOL_F32
    assert e_tr <= TOL_F32


@functools.lru_cache(maxsize=None)
def ragged_case(rec_kind):
    shape = (37, 29, 71)  # (nz, ny, nx): no dimension a multiple of any tile
    h = (10.0, 12.0, 9.0)
    vel = smooth_random(shape, seed=41)
    dt = COURANT * min(h) / 4500.0
    nt = 90
    wav = ricker(nt, dt, 25.0)
    if rec_kind == "box":
        rec = np.array([[x, y, z] for z in (2, 30) for y in range(0, 29, 7) for x in range(1, 71, 3)], dtype=np.int32)
    else:
        rng = np.random.default_rng(41)
        rec = np.stack([rng.integers(0, 71, 50), rng.integers(0, 29, 50), rng.integers(0, 37, 50)], 1).astype(np.int32)
        rec[3] = rec[7]  # a duplicate receiver
    src = (40, 13, 20)
    ref = oracle.forward(vel, h, dt, src, wav, rec, nt=nt, sponge_width=5, sponge_alpha=0.05)
    return shape, h, vel, dt, nt, wav, rec, src, ref


@pytest.mark.parametrize("rec_kind", ["box", "list"])
def test_ragged_grid_with_sponge_parity(rec_kind):
    shape, h, vel, dt, nt, wav, rec, src, ref = ragged_case(rec_kind)
    _say(f"case: ragged {shape} sponge W=5, receivers={rec_kind}")
    got = gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05)
    e_u = oracle.rel_l2(got["u"], ref["u"])
    e_tr = oracle.rel_l2(got["traces"], ref["traces"])
    # oracle's stored previous level is damped: compare g * (undamped A^{n-1})
    g = oracle.sponge_field(shape, 5, 0.05)
    e_up = oracle.rel_l2(g * got["u_prev"], ref["u_prev"])
    _say(f"rel-L2 u={e_u:.3e} g*u_prev={e_up:.3e} traces={e_tr:.3e}")
    assert e_u <= TOL_F32 and e_up <= TOL_F32 and e_tr <= TOL_F32


@pytest.mark.parametrize("rec_kind", ["box", "list"])
def test_two_steps_per_pass_is_bitwise_one_step_per_pass(rec_kind):
    """time_block = 2 (one pass advances steps n and n+1; tiles of 64 x 32
    for the first step, 56 x 24 for the second) against one step per pass in
    the fixed rule's shape: traces, A^n and the stored A^{n-1} bitwise equal,
    for an odd step count (the last step single) and an even one, for
    z-chunks from 5 planes to the whole grid, and with graph replay."""
    shape, h, vel, dt, nt, wav, rec, src, ref = ragged_case(rec_kind)
    kw = dict(sponge_width=5, sponge_alpha=0.05)
    for steps in (nt, nt - 1):
        base = gpu_run(vel, h, dt, src, wav, rec, steps, tune=False, **kw)
        for extra in (dict(), dict(zchunk=5), dict(zchunk=37), dict(graph_steps=8)):
            _say(f"case: ragged {shape} receivers={rec_kind} steps={steps} two steps per pass {extra}")
            got = gpu_run(vel, h, dt, src, wav, rec, steps, time_block=2, **kw, **extra)
            for key in ("u", "u_prev", "traces"):
                assert np.array_equal(got[key], base[key]), (key, extra)
    e_u = oracle.rel_l2(gpu_run(vel, h, dt, src, wav, rec, nt, time_block=2, **kw)["u"], ref["u"])
    _say(f"two steps per pass vs FP64 oracle: rel-L2 u={e_u:.3e}")
    assert e_u <= TOL_F32


@pytest.mark.parametrize("shape", [(5, 7, 13), (30, 26, 57), (9, 100, 64)])
def test_two_steps_per_pass_small_and_edge_grids(shape):
    """Grids smaller than one tile, fewer planes than the z reach, one tile
    wide with many in y: still the bits of one step per pass."""
    nz, ny, nx = shape
    vel = smooth_random(shape, seed=nx + ny + nz)
    dt = COURANT * 10.0 / 4500.0
    wav = ricker(33, dt, 30.0)
    src = (nx // 2, ny // 2, nz // 2)
    rec = line_receivers(nx, ny // 2, min(2, nz - 1))
    _say(f"case: two steps per pass on {shape}")
    base = gpu_run(vel, 10.0, dt, src, wav, rec, 33, tune=False)
    got = gpu_run(vel, 10.0, dt, src, wav, rec, 33, time_block=2)
    assert np.abs(base["u"]).max() > 0
    for key in ("u", "u_prev", "traces"):
        assert np.array_equal(got[key], base[key]), key


def test_two_steps_per_pass_small_workload_and_snapshot():
    """The 64^3 workload with two steps per pass: the oracle at the float32
    tolerance, and a snapshot taken after an odd step count (the buffers'
    phase mod 4 is 3) resumes bit for bit in a second context."""
    from paper_2404_04441_amd import Solver

    W, vel, wav, ref = small_case()
    _say("case: small 64^3, 200 steps, two steps per pass")
    got = gpu_run(vel, W.h, W.dt, W.src, wav, W.rec, W.nt, time_block=2)
    e_u = oracle.rel_l2(got["u"], ref["u"])
    _say(f"rel-L2 u={e_u:.3e}")
    assert e_u <= TOL_F32
    v = torch.from_numpy(vel).cuda()
    w = torch.from_numpy(wav).cuda()
    a = Solver(v, W.h, W.dt, src=W.src, rec=W.rec, time_block=2)
    tr_a = torch.zeros((W.nt, len(W.rec)), device="cuda")
    a.reset()
    a.step(71, w, tr_a)
    snap = a.save_state()
    a.step(W.nt - 71, w, tr_a)
    b = Solver(v, W.h, W.dt, src=W.src, rec=W.rec, time_block=2)
    tr_b = tr_a.clone()
    tr_b[71:] = 0
    b.load_state(snap)
    b.step(W.nt - 71, w, tr_b)
    assert torch.equal(a.read_field(0), b.read_field(0)) and torch.equal(a.read_field(1), b.read_field(1))
    assert torch.equal(tr_a, tr_b)
    a.close()
    b.close()


def test_tiling_variants_and_zchunks_are_bitwise_identical():
    """Every tile shape and z-chunk length runs the same arithmetic per node,
    so results must agree to the bit; an LDS race or halo bug breaks this."""
    from paper_2404_04441_amd import variant_count, variant_info
    from paper_2404_04441_amd._lib import WAVE_EINVAL, WaveError

    # nx = 71: shapes with 2 or 4 x nodes per lane must refuse it (EINVAL); the
    # 3D-blocked families (gmem, smem) run the same operations per node; the
    # semi-stencil family sums z in another order (checked against the oracle)
    shape, h, vel, dt, nt, wav, rec, src, ref = ragged_case("box")
    base = gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05)
    for v in range(variant_count()):
        info = variant_info(v)
        for zc in (0, 5, 16, 64):
            _say(f"case: nx=71 variant={v} {info} zchunk={zc}")
            if info["vec"] > 1:
                with pytest.raises(WaveError) as e:
                    gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05, variant=v, zchunk=zc)
                assert e.value.status == WAVE_EINVAL
                continue
            extra = dict(time_block=2) if info["family"] == 4 else {}  # the two-steps-per-pass kernel
            got = gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05, variant=v, zchunk=zc,
                          **extra)
            if info["family"] == 3:
                assert oracle.rel_l2(got["u"], ref["u"]) <= TOL_F32, (v, zc)
                assert oracle.rel_l2(got["traces"], ref["traces"]) <= TOL_F32, (v, zc)
                continue
            assert np.array_equal(got["u"], base["u"]), (v, zc)
            assert np.array_equal(got["traces"], base["traces"]), (v, zc)
    # nx = 68 (a multiple of 4, ragged against every tile width): every shape runs
    vel2 = np.ascontiguousarray(vel[:, :, :68])
    rec2 = plane_receivers(68, shape[1], 3)
    base = gpu_run(vel2, h, dt, src, wav, rec2, nt, sponge_width=5, sponge_alpha=0.05)
    ref2 = oracle.forward(vel2, h, dt, src, wav, rec2, nt=nt, sponge_width=5, sponge_alpha=0.05)
    assert oracle.rel_l2(base["u"], ref2["u"]) <= TOL_F32 and oracle.rel_l2(base["traces"], ref2["traces"]) <= TOL_F32
    for v in range(variant_count()):
        for zc in (0, 16):
            _say(f"case: nx=68 variant={v} zchunk={zc}")
            extra = dict(time_block=2) if variant_info(v)["family"] == 4 else {}
            got = gpu_run(vel2, h, dt, src, wav, rec2, nt, sponge_width=5, sponge_alpha=0.05, variant=v, zchunk=zc,
                          **extra)
            if variant_info(v)["family"] == 3:
                assert oracle.rel_l2(got["u"], ref2["u"]) <= TOL_F32, (v, zc)
                assert oracle.rel_l2(got["traces"], ref2["traces"]) <= TOL_F32, (v, zc)
                continue
            assert np.array_equal(got["u"], base["u"]), (v, zc)
            assert np.array_equal(got["traces"], base["traces"]), (v, zc)
            if variant_info(v)["family"] == 0 and zc == 0:  # the cached policy: same bits
                got = gpu_run(vel2, h, dt, src, wav, rec2, nt, sponge_width=5, sponge_alpha=0.05, variant=v,
                              cache_hint=1)
                assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"]), v


def test_tiling_query_reproduces_the_tuned_choice():
    """wave_tiling reports the configuration create settled on; passing it back
    explicitly gives the same configuration and the same bits."""
    from paper_2404_04441_amd import Solver

    shape, h, vel, dt, nt, wav, rec, src, _ = ragged_case("box")
    for nx in (71, 68):
        v = torch.from_numpy(np.ascontiguousarray(vel[:, :, :nx], dtype=np.float32)).cuda()
        r = rec[rec[:, 0] < nx]
        w = torch.from_numpy(np.ascontiguousarray(wav, dtype=np.float32)).cuda()
        outs, tilings = [], []
        for kw in ({"tune": True}, None):
            if kw is None:
                kw = dict(tilings[0])
            _say(f"case: tiling query nx={nx} {kw}")
            s = Solver(v, h, dt, src=src, rec=r, sponge_width=5, sponge_alpha=0.05, **kw)
            tilings.append(s.tiling())
            tr = s.run(nt, w)
            outs.append((s.read_field(0).cpu().numpy(), tr.cpu().numpy()))
            s.close()
        assert tilings[0] == tilings[1], tilings
        assert 1 <= tilings[0]["variant"] and tilings[0]["zchunk"] >= 1
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_tuned_shape_is_bitwise_identical():
    """Create-time tuning (the default) only chooses among shapes that compute
    the same bits as the fixed rule."""
    shape, h, vel, dt, nt, wav, rec, src, _ = ragged_case("box")
    for nx in (71, 68):
        v = np.ascontiguousarray(vel[:, :, :nx])
        r = rec[rec[:, 0] < nx]
        _say(f"case: tune=True nx={nx}")
        base = gpu_run(v, h, dt, src, wav, r, nt, sponge_width=5, sponge_alpha=0.05, tune=False)
        got = gpu_run(v, h, dt, src, wav, r, nt, sponge_width=5, sponge_alpha=0.05, tune=True)
        assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])
        _say(f"case: tune=True cache_hint=1 nx={nx}")
        got = gpu_run(v, h, dt, src, wav, r, nt, sponge_width=5, sponge_alpha=0.05, tune=True, cache_hint=1)
        assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])


def test_graph_replay_and_chunked_steps_are_bitwise_identical():
    from paper_2404_04441_amd import Solver

    shape, h, vel, dt, nt, wav, rec, src, _ = ragged_case("box")
    base = gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05)
    _say("case: graph_steps=4")
    got = gpu_run(vel, h, dt, src, wav, rec, nt, sponge_width=5, sponge_alpha=0.05, graph_steps=4)
    assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])
    _say("case: chunked wave_step 13 + 40 + rest, graph_steps=6")
    v = torch.from_numpy(vel).cuda()
    s = Solver(v, h, dt, src=src, rec=rec, sponge_width=5, sponge_alpha=0.05, graph_steps=6)
    w = torch.from_numpy(wav).cuda()
    tr = torch.zeros((nt, len(rec)), dtype=torch.float32, device="cuda")
    for rep in range(2):  # the second pass replays graphs captured in the first
        s.reset()
        s.step(13, w, tr)
        s.step(40, w, tr)
        s.step(nt - 53, w, tr)
        assert s.time_index() == nt
        torch.cuda.synchronize()
        assert np.array_equal(s.read_field(0).cpu().numpy(), base["u"]), rep
        assert np.array_equal(tr.cpu().numpy(), base["traces"]), rep
    s.close()


@pytest.mark.parametrize("shape,src", [((1, 1, 1), (0, 0, 0)), ((1, 1, 9), (4, 0, 0)), ((6, 1, 1), (0, 0, 3)),
                                       ((2, 3, 4), (3, 2, 1)), ((9, 70, 65), (64, 69, 8)),
                                       # 4 x nodes per lane: two active lanes; one row; a 4-column second tile
                                       ((3, 2, 8), (5, 1, 1)), ((5, 1, 12), (11, 0, 2)), ((4, 9, 260), (258, 8, 0)),
                                       # 2 x nodes per lane (nx even, not a multiple of 4)
                                       ((7, 5, 18), (17, 4, 6))])
def test_degenerate_and_edge_grids(shape, src):
    nz, ny, nx = shape
    vel = np.full(shape, 2500.0, dtype=np.float32)
    vel[..., : max(1, nx // 2)] = 1800.0
    h, dt, nt = 10.0, COURANT * 10.0 / 4500.0, 25
    wav = ricker(nt, dt, 40.0, t0=0.0)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rec = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.int32)[:4096]
    _say(f"case: edge grid {shape} src={src}")
    ref = oracle.forward(vel, h, dt, src, wav, rec, nt=nt)
    got = gpu_run(vel, h, dt, src, wav, rec, nt)
    assert oracle.rel_l2(got["u"], ref["u"]) <= TOL_F32
    assert oracle.rel_l2(got["traces"], ref["traces"]) <= TOL_F32


def test_no_source_no_receivers_stays_zero():
    vel = np.full((20, 21, 22), 3000.0, dtype=np.float32)
    got = gpu_run(vel, 10.0, 1e-4, None, np.zeros(1, np.float32), None, 10)
    assert not got["u"].any() and got["traces"] is None


def test_mirror_symmetry_and_linearity_mid_size():
    """A velocity symmetric about the source gives a field symmetric to the
    bit (a + b == b + a).  Doubling the wavelet doubles the field up to
    rounding: x2 is exact except in the underflowing tail ahead of the front,
    whose perturbations can flip near-tie roundings that then propagate."""
    n = (65, 97, 129)  # (nz, ny, nx), all odd
    zc, yc, xc = (k // 2 for k in n)
    zz, yy, xx = np.meshgrid(*(np.arange(k) for k in n), indexing="ij")
    r2 = ((xx - xc) / 40.0) ** 2 + ((yy - yc) / 30.0) ** 2 + ((zz - zc) / 20.0) ** 2
    vel = (2000.0 + 1500.0 * np.exp(-r2)).astype(np.float32)
    dt = COURANT * 10.0 / 3500.0
    nt = 120
    wav = ricker(nt, dt, 15.0)
    _say("case: mirror symmetry 129x97x65 with sponge")
    a = gpu_run(vel, 10.0, dt, (xc, yc, zc), wav, None, nt, sponge_width=8, sponge_alpha=0.03)["u"]
    assert np.abs(a).max() > 0
    assert np.array_equal(a, a[:, :, ::-1]) and np.array_equal(a, a[:, ::-1, :]) and np.array_equal(a, a[::-1])
    b = gpu_run(vel, 10.0, dt, (xc, yc, zc), 2 * wav, None, nt, sponge_width=8, sponge_alpha=0.03)["u"]
    assert np.abs(b - 2 * a).max() <= 1e-6 * np.abs(2 * a).max()


def test_full_size_512_sampled_one_step():
    """The 512^3 workload in the launch configuration the benchmark times:
    after 40 steps, one more GPU step is checked node by node against the
    oracle's one-step formula at 3000 sampled nodes (edges, sponge, tile
    borders, the source and random interior), and its trace row against the
    field on the receiver plane."""
    from paper_2404_04441_amd import Solver

    W = workload("large")
    vel = W.velocity()
    wav = W.wavelet()
    _say("case: 512^3 large workload, sampled step check")
    v = torch.from_numpy(vel).cuda()
    s = Solver(v, W.h, W.dt, src=W.src, rec=W.rec, sponge_width=W.sponge_width, sponge_alpha=W.sponge_alpha)
    w = torch.from_numpy(wav).cuda()
    tr = torch.zeros((W.nt, len(W.rec)), dtype=torch.float32, device="cuda")
    s.reset()
    s.step(40, w, tr)
    A_n = s.read_field(0).cpu().numpy()
    A_nm1 = s.read_field(1).cpu().numpy()
    s.step(1, w, tr)
    A_np1 = s.read_field(0).cpu().numpy()
    row = tr[40].cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    n = 512
    rng = np.random.default_rng(99)
    pts = [rng.integers(0, n, size=(1500, 3))]
    edge = np.array([0, 1, 3, 4, 19, 20, 21, 63, 64, 65, 255, 256, 447, 448, 491, 492, 507, 508, 510, 511])
    pts.append(np.stack([rng.choice(edge, 1500), rng.choice(edge, 1500), rng.choice(edge, 1500)], 1))
    pts.append(np.array([W.src]))
    pts = np.concatenate(pts)
    ref = oracle.step_at(pts, A_n, A_nm1, vel, W.h, W.dt, src=W.src, s_n=float(wav[40]),
                         sponge_width=W.sponge_width, sponge_alpha=W.sponge_alpha)
    got = A_np1[pts[:, 2], pts[:, 1], pts[:, 0]]
    scale = np.abs(A_np1).max()
    err = np.abs(got - ref).max() / scale
    _say(f"max sampled error / max|A| = {err:.3e}")
    assert scale > 0 and err <= 1e-6
    assert np.array_equal(row, A_np1[0].ravel())


class _Gathered:
    """A few nodes of a device array, gathered to the host: indexed [z, y, x]
    like the array itself, for the oracle's pointwise step."""

    def __init__(self, shape, table):
        self.shape = shape
        self._t = table

    def __getitem__(self, idx):
        return self._t[tuple(int(i) for i in idx)]


def _random_state_one_step(W, vel_dev, seed, edge, **solver_kw):
    """A^n and the stored A^{n-1} set to seeded random normal fields, so that
    every tile edge and z-chunk boundary carries data; one GPU step from that
    state is checked against the oracle's one-step formula at sampled nodes
    (random, and on tile / chunk / sponge edges), and its trace row against
    the new field at the receivers."""
    from paper_2404_04441_amd import Solver

    dev = vel_dev.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    A_n = torch.randn(W.shape, generator=gen, device=dev)
    A_nm1 = torch.randn(W.shape, generator=gen, device=dev)
    s = Solver(vel_dev, W.h, W.dt, src=W.src, rec=W.rec, sponge_width=W.sponge_width,
               sponge_alpha=W.sponge_alpha, **solver_kw)
    wav = torch.from_numpy(W.wavelet()).to(dev)
    tr = torch.zeros((1, len(W.rec)), dtype=torch.float32, device=dev)
    s.reset()
    s.write_field(0, A_n)
    s.write_field(1, A_nm1)
    s.step(1, wav, tr)
    A_np1 = s.read_field(0)
    tiling = s.tiling()
    s.close()
    from paper_2404_04441_amd import variant_info

    info = variant_info(tiling["variant"])
    _say(f"tiling {tiling} {info}")
    nz, ny, nx = W.shape
    # nodes on both sides of every tile edge and z-chunk boundary of this configuration
    tx = 64 * info["vec"] if info["family"] in (0, 3) else 64
    ty = info["by"] * info["ry"] if info["family"] in (0, 3) else info["by"]
    tz = tiling["zchunk"]

    def around(step, n):
        k = np.arange(step, n, step)
        return np.concatenate([k - 1, k, edge[edge < n]])

    ex, ey, ez = around(tx, nx), around(ty, ny), around(tz, nz)
    rng = np.random.default_rng(seed)
    pts = [np.stack([rng.integers(0, nx, 1500), rng.integers(0, ny, 1500), rng.integers(0, nz, 1500)], 1)]
    pts.append(np.stack([rng.choice(ex, 3000), rng.choice(ey, 3000), rng.choice(ez, 3000)], 1))
    pts.append(np.array([W.src]))
    pts = np.concatenate(pts)
    offs = [(0, 0, 0)] + [o for m in range(1, 5) for o in
                          ((m, 0, 0), (-m, 0, 0), (0, m, 0), (0, -m, 0), (0, 0, m), (0, 0, -m))]
    need = sorted({(z + dz, y + dy, x + dx) for x, y, z in pts for dx, dy, dz in offs
                   if 0 <= x + dx < nx and 0 <= y + dy < ny and 0 <= z + dz < nz})
    idx = torch.from_numpy(np.array(need, dtype=np.int64)).to(dev)
    tables = [dict(zip(need, t[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy().tolist()))
              for t in (A_n, A_nm1, vel_dev)]
    an, ap, vv = (_Gathered(W.shape, t) for t in tables)
    ref = oracle.step_at(pts, an, ap, vv, W.h, W.dt, src=W.src, s_n=float(wav[0]), sponge_width=W.sponge_width,
                         sponge_alpha=W.sponge_alpha)
    p = torch.from_numpy(pts.astype(np.int64)).to(dev)
    got = A_np1[p[:, 2], p[:, 1], p[:, 0]].double().cpu().numpy()
    scale = float(A_np1.abs().max())
    err = np.abs(got - ref).max() / scale
    _say(f"max sampled error / max|A| = {err:.3e} over {len(pts)} nodes")
    assert scale > 0 and err <= 1e-6
    r = torch.from_numpy(np.asarray(W.rec, dtype=np.int64)).to(dev)
    assert torch.equal(tr[0], A_np1[r[:, 2], r[:, 1], r[:, 0]])


def test_full_size_512_random_state_one_step():
    """The 512^3 workload (sponge, source, receiver plane) in the benchmark's
    configuration (the fixed rule's shape and z-chunk)."""
    W = workload("large")
    _say("case: 512^3 large workload, one step from a random state")
    vel = torch.from_numpy(W.velocity()).cuda()
    edge = np.array([0, 1, 3, 4, 19, 20, 21, 63, 64, 65, 255, 256, 257, 260, 261, 262, 447, 448, 491, 492, 507,
                     508, 510, 511])
    _random_state_one_step(W, vel, 512, edge, tune=False)


def test_full_size_1024_random_state_one_step():
    """The 1024^3 workload (smooth random model on the device, Dirichlet, line
    of 1024 receivers) in the configuration the benchmark times for it
    (create-time tuning; z-chunks capped so a workgroup's buffers span less
    than 2 GiB)."""
    from synth.velocity import smooth_random_torch

    W = workload("precision")
    _say("case: 1024^3 precision workload, one step from a random state")
    vel = smooth_random_torch(W.shape, seed=3, device=torch.device("cuda"))
    edge = np.array([0, 1, 3, 4, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 459, 460, 461, 511, 512, 513, 767,
                     768, 919, 920, 921, 1019, 1020, 1022, 1023])
    _random_state_one_step(W, vel, 1024, edge)
    del vel
    torch.cuda.empty_cache()
