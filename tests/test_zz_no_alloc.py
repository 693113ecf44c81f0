"""wave_create_static, the entry point for callers that cannot allocate
device memory, against wave_create on the same inputs: two calls in a row
(the second on a smaller grid, so the static array still holds the first
call's larger contents), each bitwise equal to the caller-workspace path
(same kernels and tile configuration: the fixed rule, tuning off on both)."""
import ctypes

import numpy as np
import pytest

from synth import COURANT, ricker, smooth_random
from synth.workloads import line_receivers, plane_receivers

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def _params(L, lib, shape, h, dt, src, rec, storage, sponge):
    nz, ny, nx = shape
    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    p.nx, p.ny, p.nz = nx, ny, nz
    p.dx = p.dy = p.dz = h
    p.dt = dt
    p.sponge_width, p.sponge_alpha = sponge, 0.05
    p.storage = storage
    p.src[0], p.src[1], p.src[2] = src
    p.nrec = len(rec)
    p.rec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.tune = 0
    return p


def _run(static, p, vel, wav, nt, nrec, shape):
    from paper_2404_04441_amd import _lib as L

    lib = L.lib()
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    ws = None
    if static:
        L.check(lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream.cuda_stream, ctypes.byref(h)),
                "wave_create_static")
    else:
        nb = ctypes.c_size_t()
        L.check(lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)), "wave_workspace_bytes")
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (ws.data_ptr() + 255) // 256 * 256
        L.check(lib.wave_create(ctypes.byref(p), vel.data_ptr(), ptr, nb.value, stream.cuda_stream, ctypes.byref(h)),
                "wave_create")
    traces = torch.empty((nt, nrec), dtype=torch.float32, device="cuda")
    field = torch.empty(shape, dtype=torch.float32, device="cuda")
    L.check(lib.wave_run(h, nt, wav.data_ptr(), traces.data_ptr()), "wave_run")
    L.check(lib.wave_read_field(h, 0, field.data_ptr()), "wave_read_field")
    L.check(lib.wave_destroy(h), "wave_destroy")
    torch.cuda.synchronize()
    del ws
    return traces.cpu().numpy(), field.cpu().numpy()


def test_static_workspace_matches_caller_workspace_twice():
    from paper_2404_04441_amd import _lib as L

    lib = L.lib()
    h = 10.0
    cases = [
        # float32, sponge, a receiver plane (fused receivers), 96 x 80 x 72
        dict(shape=(72, 80, 96), src=(48, 40, 30), rec=plane_receivers(96, 80, 5), storage=L.WAVE_F32, sponge=6,
             nt=90, seed=81),
        # smaller: 16-bit storage, Dirichlet, a receiver line, 40 x 36 x 30
        dict(shape=(30, 36, 40), src=(20, 18, 15), rec=line_receivers(40, 18, 4), storage=L.WAVE_F16, sponge=0,
             nt=60, seed=82),
    ]
    for c in cases:
        _say(f"case: static vs caller workspace {c['shape']} storage {c['storage']} nt {c['nt']}")
        vel_np = smooth_random(c["shape"], seed=c["seed"])
        dt = COURANT * h / 4500.0
        vel = torch.from_numpy(vel_np).cuda()
        wav = torch.from_numpy(ricker(c["nt"], dt, 25.0)).cuda()
        rec = np.ascontiguousarray(c["rec"], dtype=np.int32)
        p = _params(L, lib, c["shape"], h, dt, c["src"], rec, c["storage"], c["sponge"])
        ref_tr, ref_u = _run(False, p, vel, wav, c["nt"], len(rec), c["shape"])
        got_tr, got_u = _run(True, p, vel, wav, c["nt"], len(rec), c["shape"])
        assert np.abs(ref_u).max() > 0 and np.abs(ref_tr).max() > 0
        assert np.array_equal(got_tr, ref_tr) and np.array_equal(got_u, ref_u)


def test_static_workspace_limits():
    """One static context per device at a time; graph replay refused;
    workspaces beyond the static array's size refused."""
    from paper_2404_04441_amd import _lib as L

    lib = L.lib()
    shape = (20, 20, 20)
    dt = COURANT * 10.0 / 4500.0
    vel = torch.from_numpy(smooth_random(shape, seed=83)).cuda()
    rec = np.zeros((0, 3), dtype=np.int32)
    p = _params(L, lib, shape, 10.0, dt, (10, 10, 10), rec, L.WAVE_F32, 0)
    stream = torch.cuda.current_stream().cuda_stream
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    L.check(lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream, ctypes.byref(a)), "first")
    assert lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream, ctypes.byref(b)) == L.WAVE_ESTATE
    L.check(lib.wave_destroy(a), "destroy")
    L.check(lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream, ctypes.byref(b)), "again")
    L.check(lib.wave_destroy(b), "destroy")
    p.graph_steps = 10
    assert lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream, ctypes.byref(b)) == L.WAVE_EINVAL
    p.graph_steps = 0
    p.nx = p.ny = p.nz = 256
    assert lib.wave_create_static(ctypes.byref(p), vel.data_ptr(), stream, ctypes.byref(b)) == L.WAVE_ENOSPC
