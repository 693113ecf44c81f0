"""GPU parity of the CPML boundary against the FP64 oracle (through the C ABI).

The oracle's CPML is pinned on the CPU (tests/test_oracle_cpml.py: textbook
weights, the undamped limit, absorption against a large domain).  Here the
GPU's three-part step (memory-variable update, fused step, boundary
correction) must match it within the float32 tolerance of the plain step,
on a ragged grid with receivers inside and outside the layers.
"""
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


def test_cpml_shapes_and_replay_are_bitwise_identical():
    from paper_2404_04441_amd import variant_count, variant_info

    vel, h, dt, wav, rec, src, W, nt = _case(nt=60)
    base = _gpu(vel, h, dt, wav, rec, src, W, nt)
    for v in range(variant_count()):
        info = variant_info(v)
        if info["family"] not in (0,) or vel.shape[2] % info["vec"]:
            continue
        _say(f"case: CPML variant {v} {info}")
        got = _gpu(vel, h, dt, wav, rec, src, W, nt, variant=v)
        assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"]), v
    _say("case: CPML graph replay")
    got = _gpu(vel, h, dt, wav, rec, src, W, nt, graph_steps=6)
    assert np.array_equal(got["u"], base["u"]) and np.array_equal(got["traces"], base["traces"])


def test_cpml_layer_as_thick_as_half_the_grid():
    vel, h, dt, wav, rec, src, W, nt = _case(shape=(20, 24, 28), W=10, nt=50)
    ref = forward_cpml(vel, h, dt, src, wav, rec, nt, width=W, f0=30.0)
    got = _gpu(vel, h, dt, wav, rec, src, W, nt)
    e_u = oracle.rel_l2(got["u"], ref["u"])
    _say(f"case: W = nz/2: rel-L2 field {e_u:.3e}")
    assert e_u <= TOL
