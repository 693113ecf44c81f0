"""Serving on the GPU: each shot's traces are the same alone and in the mix.

Shots run on separate streams through captured-graph chunks and share the
device; no shot's arithmetic depends on another's, so the comparison is
bitwise.  The float32 shots are also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2404_04441_amd.serve import GpuBackend, ShotRequest, ShotServer, summarize
from synth import COURANT
from synth.velocity import layered_profile
from synth.workloads import line_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests():
    shapes = [(48, 48, 48), (40, 56, 64), (64, 64, 64), (33, 47, 71)]
    out = []
    for i in range(10):
        nz, ny, nx = shapes[i % 4]
        # the first three arrive together, so at least two run at once whatever the device's speed
        out.append(ShotRequest(id=i, arrival=0.0 if i < 3 else 0.004 * i, shape=(nz, ny, nx), nt=60 + 11 * i,
                               storage="f16" if i % 3 == 2 else "f32", h=10.0, dt=COURANT * 10.0 / 4500.0,
                               src=(nx // 2, ny // 2, 4), rec=line_receivers(nx, ny // 2, 3), f0=25.0,
                               sponge_width=6, sponge_alpha=0.05, velocity=layered_profile(nz, 5000 + i)))
    return out


@pytest.mark.parametrize("lanes", [0, 2])
def test_each_shot_is_the_same_alone_and_in_the_mix(lanes):
    reqs = _requests()
    print(f"case: 10 shots mixed, 4 slots, graph chunks, lanes {lanes}", flush=True)
    server = ShotServer(GpuBackend(graph_steps=10, lanes=lanes), budget_bytes=4 << 30, max_slots=4, chunk_steps=40)
    mixed = server.run(reqs)
    summary = summarize(mixed, reqs, server.elapsed)
    print(summary, "max concurrent", server.max_concurrent, flush=True)
    assert summary["done"] == len(reqs) and server.max_concurrent >= 2
    for r in reqs:
        print(f"case: shot {r.id} alone", flush=True)
        alone = ShotServer(GpuBackend(graph_steps=10), budget_bytes=4 << 30, max_slots=1, chunk_steps=40)
        r0 = ShotRequest(**{**r.__dict__, "arrival": 0.0})
        res = alone.run([r0])[r.id]
        assert res.status == "done"
        assert torch.equal(res.traces, mixed[r.id].traces), r.id
        if r.storage == "f32":
            vel = np.broadcast_to(r.velocity[:, None, None], r.shape).astype(np.float32)
            from synth import ricker
            ref = oracle.forward(vel, r.h, r.dt, r.src, ricker(r.nt, r.dt, r.f0, r.t0), r.rec, nt=r.nt,
                                 sponge_width=r.sponge_width, sponge_alpha=r.sponge_alpha)
            e = oracle.rel_l2(res.traces.cpu().numpy(), ref["traces"])
            print(f"shot {r.id} f32 traces vs oracle: {e:.2e}", flush=True)
            assert e <= 1e-5


def test_failures_do_not_stop_the_server():
    reqs = _requests()[:3]
    bad = ShotRequest(**{**reqs[0].__dict__, "id": 99, "dt": 1.0})  # far above the stability limit
    server = ShotServer(GpuBackend(), budget_bytes=4 << 30, max_slots=2, chunk_steps=40)
    res = server.run(reqs + [bad])
    assert res[99].status == "failed" and "stability" in res[99].error
    assert all(res[r.id].status == "done" for r in reqs)
