"""Shot snapshots: saving the state after n steps and resuming it (in the same
context or in a fresh one with the same parameters) continues bit for bit,
for float32 with a sponge, 16-bit storage and the CPML boundary."""
import numpy as np
import pytest

from synth import COURANT, ricker, smooth_random

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("kind", ["f32-sponge", "f16", "bf16", "f32-cpml"])
def test_snapshot_resumes_bit_for_bit(kind):
    from paper_2404_04441_amd import Solver
    from paper_2404_04441_amd._lib import WAVE_EINVAL, WaveError

    shape = (34, 29, 40)
    h = 10.0
    vel = torch.from_numpy(smooth_random(shape, seed=91)).cuda()
    dt = COURANT * h / 4500.0
    nt = 70
    wav = torch.from_numpy(ricker(nt, dt, 30.0)).cuda()
    rec = np.array([[x, 14, 3] for x in range(0, 40, 2)], dtype=np.int32)
    kw = dict(src=(20, 14, 16), rec=rec)
    if kind == "f32-cpml":
        kw.update(cpml_width=6, cpml_f0=30.0)
    else:
        kw.update(sponge_width=5, sponge_alpha=0.05, storage=kind.split("-")[0])
    _say(f"case: snapshot {kind}")
    s = Solver(vel, h, dt, **kw)
    tr = torch.zeros((nt, len(rec)), device="cuda")
    s.reset()
    s.step(40, wav, tr)
    snap = s.save_state()
    s.step(30, wav, tr)
    ref_u = s.read_field(0).clone()
    ref_tr = tr[40:].clone()
    # same context
    s.load_state(snap)
    assert s.time_index() == 40
    tr2 = torch.zeros_like(tr)
    s.step(30, wav, tr2)
    assert torch.equal(s.read_field(0), ref_u) and torch.equal(tr2[40:], ref_tr)
    s.close()
    # a fresh context with the same parameters
    s2 = Solver(vel, h, dt, **kw)
    s2.load_state(snap)
    tr3 = torch.zeros_like(tr)
    s2.step(30, wav, tr3)
    assert torch.equal(s2.read_field(0), ref_u) and torch.equal(tr3[40:], ref_tr)
    s2.close()
    # a context with another grid refuses it
    s3 = Solver(vel[:-1].contiguous(), h, dt, **kw)
    with pytest.raises(WaveError) as e:
        s3.load_state(snap)
    assert e.value.status == WAVE_EINVAL
    s3.close()
