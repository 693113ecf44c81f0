"""GPU parity of the CPML boundary against the FP64 oracle (through the C ABI).

The oracle's CPML is pinned on the CPU (tests/test_oracle_cpml.py: textbook
weights, the undamped limit, absorption against a large domain).  Here the
GPU step with CPML (memory-variable pass; the step with the x part of the
boundary terms fused in, then a correction pass for the y and z parts; or,
for shapes without a fused kernel, the plain step and a correction pass for
all three) must match it within the float32 tolerance of the plain step, on
ragged grids with receivers inside and outside the layers.
"""
import functools

import numpy as np
import pytest

import oracle
from oracle.cpml import forward_cpml
from synth import COURANT, ricker, smooth_random

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


def _say(*a):
    print(*a, flush=True)


def _case(shape=(33, 30, 44), W=6, nt=120):
    h = (10.0, 11.0, 9.0)
    vel = smooth_random(shape, seed=77)
    dt = COURANT * min(h) / 4500.0
    wav = ricker(nt, dt, 30.0)
    nz, ny, nx = shape
    rec = np.array([[x, y, z] for z in (2, 16) for y in range(1, ny, 5) for x in range(0, nx, 3)], dtype=np.int32)
    src = (nx // 2, ny // 2, nz // 2 - 3)
    return vel, h, dt, wav, rec, src, W, nt


def _gpu(vel, h, dt, wav, rec, src, W, nt, f0=30.0, **kw):
    from paper_2404_04441_amd import Solver

    s = Solver(torch.from_numpy(vel).cuda(), h, dt, src=src, rec=rec, cpml_width=W, cpml_f0=f0, **kw)
    tr = s.run(nt, torch.from_numpy(wav).cuda())
    out = {"u": s.read_field(0).cpu().numpy(), "traces": tr.cpu().numpy()}
    torch.cuda.synchronize()
    s.close()
    return out


def test_cpml_matches_oracle():
    vel, h, dt, wav, rec, src, W, nt = _case()
    _say(f"case: CPML W={W} grid {vel.shape} {nt} steps")
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    got = _gpu(vel, h, dt, wav, rec, src, W, nt)
    e_u, e_t = oracle.rel_l2(got["u"], ref["u"]), oracle.rel_l2(got["traces"], ref["traces"])
    _say(f"rel-L2 field {e_u:.3e} traces {e_t:.3e}")
    assert np.abs(ref["zeta"][0]).max() > 0  # the layers were reached
    assert e_u <= TOL and e_t <= TOL


def _fused(info):
    """Shapes whose step kernel applies the x part of the CPML terms itself
    (2.5D shapes with at most two rows per wavefront and four nodes per thread)."""
    return info["family"] == 0 and info["ry"] <= 2 and info["ry"] * info["vec"] <= 4


def test_cpml_shapes_and_replay():
    """Fused shapes: bitwise identical to each other and under graph replay.
    Shapes that take the separate correction pass: within the tolerance of
    the oracle."""
    from paper_2404_04441_amd import variant_count, variant_info

    vel, h, dt, wav, rec, src, W, nt = _case(nt=60)
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    base = _gpu(vel, h, dt, wav, rec, src, W, nt)
    assert oracle.rel_l2(base["u"], ref["u"]) <= TOL
    nfused = 0
    for v in range(1, variant_count()):
        info = variant_info(v)
        if vel.shape[2] % info["vec"] or info["family"] == 4:  # family 4 (two steps per pass) has no CPML
            continue
        _say(f"case: CPML variant {v} {info} fused={_fused(info)}")
        got = _gpu(vel, h, dt, wav, rec, src, W, nt, variant=v)
        if _fused(info):
            nfused += 1
            assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"]), v
        else:
            e_u, e_t = oracle.rel_l2(got["u"], ref["u"]), oracle.rel_l2(got["traces"], ref["traces"])
            assert e_u <= TOL and e_t <= TOL, (v, e_u, e_t)
    assert nfused >= 3
    _say("case: CPML with create-time tuning (fused shapes only)")
    got = _gpu(vel, h, dt, wav, rec, src, W, nt, tune=1)
    assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])
    _say("case: CPML graph replay")
    got = _gpu(vel, h, dt, wav, rec, src, W, nt, graph_steps=6)
    assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])


def test_cpml_tile_edges_inside_the_layers():
    """nx = 264 with 4-node lanes: two 256-wide tiles, and the right x layer
    (W = 11: columns 253 .. 263) starts just before the second tile at 256, so
    psi_x crosses the tile edge through the x halo; odd W also splits lanes'
    columns between layer and interior.  Checked on the whole field and on
    the crop around the edge, where the source sits."""
    vel, h, dt, wav, rec, src, W, nt = _case(shape=(24, 24, 264), W=11, nt=70)
    src = (252, 10, 11)
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    got = _gpu(vel, h, dt, wav, rec, src, W, nt)
    e_u, e_t = oracle.rel_l2(got["u"], ref["u"]), oracle.rel_l2(got["traces"], ref["traces"])
    e_c = oracle.rel_l2(got["u"][:, :, 236:], ref["u"][:, :, 236:])
    _say(f"case: CPML tile edges in the layers: rel-L2 field {e_u:.3e} crop {e_c:.3e} traces {e_t:.3e}")
    assert np.abs(ref["psi"][0][:, :, 250:258]).max() > 0
    assert e_u <= TOL and e_t <= TOL and e_c <= TOL


@pytest.mark.parametrize("nx", [45, 46])
def test_cpml_narrow_lanes(nx):
    """Odd nx (one node per lane) and nx = 2 mod 4 (two nodes per lane)."""
    vel, h, dt, wav, rec, src, W, nt = _case(shape=(26, 21, nx), W=7, nt=70)
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    got = _gpu(vel, h, dt, wav, rec, src, W, nt)
    e_u, e_t = oracle.rel_l2(got["u"], ref["u"]), oracle.rel_l2(got["traces"], ref["traces"])
    _say(f"case: CPML nx={nx}: rel-L2 field {e_u:.3e} traces {e_t:.3e}")
    assert e_u <= TOL and e_t <= TOL


def test_cpml_layer_as_thick_as_half_the_grid():
    vel, h, dt, wav, rec, src, W, nt = _case(shape=(20, 24, 28), W=10, nt=50)
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    got = _gpu(vel, h, dt, wav, rec, src, W, nt)
    e_u = oracle.rel_l2(got["u"], ref["u"])
    _say(f"case: W = nz/2: rel-L2 field {e_u:.3e}")
    assert e_u <= TOL


@functools.lru_cache(maxsize=None)
def _large_velocity():
    from synth import workload

    return workload("large").velocity()


@pytest.mark.parametrize("corner", ["low", "high"])
def test_cpml_full_size_light_cone(corner):
    """The 512^3 CPML configuration the bench times (W = 20, R = 1e-3,
    f0 = 15 Hz, the same create-time choice of fused shape), with the source
    inside a corner's layers, checked against the oracle at full size.

    In the layers a step reaches at most 8 nodes along an axis (D1 of psi,
    which is D1 of A), so after k = 6 steps the field is zero beyond 48 nodes
    of the source.  The oracle runs on the 96^3 cube at that corner (profiles
    from the full grid's v_max; the cube's inner faces and their layers lie
    beyond the reach), which gives the exact reference inside the cube; every
    node outside the cube must be exactly zero on the GPU."""
    from paper_2404_04441_amd import Solver
    from synth import workload

    W = workload("large")
    vel = _large_velocity()
    nz, ny, nx = vel.shape
    k, C = 6, 96
    if corner == "low":
        src = (6, 7, 5)
        sl = (slice(0, C),) * 3
        src_c = src
    else:
        src = (nx - 7, ny - 6, nz - 8)
        sl = (slice(nz - C, nz), slice(ny - C, ny), slice(nx - C, nx))
        src_c = (src[0] - (nx - C), src[1] - (ny - C), src[2] - (nz - C))
    wav = W.wavelet(k)
    _say(f"case: CPML 512^3 light cone, {corner} corner, source {src}, {k} steps")
    s = Solver(torch.from_numpy(vel).cuda(), W.h, W.dt, src=src, rec=None, cpml_width=W.sponge_width, cpml_f0=W.f0)
    s.run(k, torch.from_numpy(wav).cuda())
    u = s.read_field(0)
    crop = u[sl].cpu().numpy()
    u[sl] = 0
    outside = float(u.abs().max())
    torch.cuda.synchronize()
    s.close()
    ref = forward_cpml(np.ascontiguousarray(vel[sl]), W.h, W.dt, src_c, wav, np.zeros((0, 3), dtype=np.int32), k,
                       width=W.sponge_width, f0=W.f0, vmax=float(vel.max()))
    assert np.abs(ref["psi"][0]).max() > 0 and np.abs(ref["zeta"][2]).max() > 0  # the layers are active
    e = oracle.rel_l2(crop, ref["u"])
    _say(f"rel-L2 in the corner cube {e:.3e}, max outside {outside:.1e}")
    assert outside == 0.0
    assert e <= TOL
