#!/usr/bin/env python3
"""Benchmark: the fused 8th-order acoustic stencil on one MI355X.

One benchmark "step" is one whole forward shot of the 512^3 workload: reset
(zero both wavefields) then 1000 fused time steps with the 20-node sponge, the
Ricker point source and the 512x512 receiver plane sampled every step.  All
inputs (velocity, wavelet) are resident in HBM before timing starts.

value = grid points x time steps / wall time (Gpts/s) over the timed shots.
roofline: algorithmic bytes of one fused step (16 B per point: read A^n,
A^{n-1}, m; write A^{n+1}) / the step kernel's average duration, measured with
HIP events on the solver's stream over a run of step kernels only.
cpu_baseline: the FP64 NumPy oracle timed on the host for one time step of
the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
# algorithmic bytes per point-step: float32 reads A^n, A^{n-1}, m and writes A^{n+1};
# 16-bit storage reads A^n, V^n (2 B each) and m (4 B, or 2 B as 16-bit codes),
# writes A^{n+1} and V^{n+1}
BYTES_PER_POINT = {"f32": 16, "f16": 12, "bf16": 12, "f16_m16": 10, "bf16_m16": 10}
# the survey's figure for a 16-bit storage step (two 16-bit levels read, one
# written, float32 m): each 16-bit form is also quoted against it
SURVEY_16BIT_BYTES = 10


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("step_kernels.h", "step_f32.hip", "wave_internal.h"):
        with open(os.path.join(ROOT, "paper_2404_04441_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, tiling: dict):
    """HBM bytes per step kernel from committed rocprofv3 counter runs, only
    if they were taken on the current kernel source and the same step
    configuration (variant, z-chunk, cache policy)."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_large_{storage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sha") != kernel_source_hash() or rec.get("tiling") != tiling:
        return None
    return rec.get("bytes_per_launch")


def _oracle_steps(args):
    """Seconds for `steps` oracle steps of an n^3 serving shot (a worker of
    the all-core sample; imports inside, so it runs in a fresh process)."""
    n, steps, seed = args
    import time as _t

    import oracle
    from synth import COURANT, ricker
    from synth.velocity import layered_profile

    vel = np.broadcast_to(layered_profile(n, seed)[:, None, None], (n, n, n)).astype(np.float32)
    dt = COURANT * 10.0 / 4500.0
    rec = np.array([[x, n // 2, 4] for x in range(n)])
    t0 = _t.perf_counter()
    oracle.forward(vel, 10.0, dt, (n // 2, n // 2, 4), ricker(steps, dt, 15.0), rec, nt=steps, sponge_width=20,
                   sponge_alpha=0.015)
    return _t.perf_counter() - t0


def cpu_baseline(W, vel):
    """The oracle as it is (NumPy, FP64, one thread per process), timed on
    bounded samples: the headline value is enough time steps of the full
    512^3 workload for ~10 s; beside it the whole 64^3 x 200 workload, the
    whole 128^3 x 500 crop of the 1024^3 workload, 10 forward steps of the
    256^3 gradient workload, and an all-core estimate of serving shots/s (one
    process per core, each a few steps of a 128^3 serving shot, extrapolated
    to the stream's mean of 1250 steps)."""
    import math
    from concurrent.futures import ProcessPoolExecutor

    import oracle
    from synth import workload

    def timed(steps):
        wav = W.wavelet(steps)
        t0 = time.perf_counter()
        oracle.forward(vel, W.h, W.dt, W.src, wav, W.rec, nt=steps, sponge_width=W.sponge_width,
                       sponge_alpha=W.sponge_alpha)
        return time.perf_counter() - t0

    t1 = timed(1)
    steps = 1 if t1 >= 10.0 else min(8, math.ceil(10.0 / t1))
    t = timed(steps) if steps > 1 else t1
    out = {"value": round(W.npts * steps / t / 1e9, 5), "unit": "Gpts/s", "cores": 1, "kind": "oracle",
           "sample": f"{steps} time steps of the {W.name} workload (sponge, source, 512x512 receivers), "
                     f"FP64 NumPy oracle, single thread, {t:.1f} s; host reports {os.cpu_count()} CPUs"}
    S = workload("small")
    t0 = time.perf_counter()
    oracle.forward(S.velocity(), S.h, S.dt, S.src, S.wavelet(), S.rec, nt=S.nt)
    ts = time.perf_counter() - t0
    out["small_full_run"] = {"workload": f"{S.name} x {S.nt} steps (whole run)", "seconds": round(ts, 2),
                             "gpts_per_s": round(S.npts * S.nt / ts / 1e9, 5), "cores": 1}
    C = workload("precision_crop")
    t0 = time.perf_counter()
    oracle.forward(C.velocity(), C.h, C.dt, C.src, C.wavelet(), C.rec, nt=C.nt)
    tc = time.perf_counter() - t0
    out["crop_full_run"] = {"workload": f"{C.name} x {C.nt} steps (whole run)", "seconds": round(tc, 2),
                            "gpts_per_s": round(C.npts * C.nt / tc / 1e9, 5), "cores": 1}
    G = workload("gradient")
    gsteps = 10
    t0 = time.perf_counter()
    oracle.forward(G.velocity(), G.h, G.dt, G.src, G.wavelet(gsteps), G.rec, nt=gsteps)
    tg = time.perf_counter() - t0
    out["gradient_workload_forward"] = {
        "workload": f"{G.name}: {gsteps} forward steps (the gradient also runs the adjoint)",
        "s_per_step": round(tg / gsteps, 4), "gpts_per_s": round(G.npts * gsteps / tg / 1e9, 5), "cores": 1}
    procs = max(1, min(16, os.cpu_count() or 1))
    per = 4
    t0 = time.perf_counter()
    with ProcessPoolExecutor(procs) as pool:
        secs = list(pool.map(_oracle_steps, [(128, per, 5000 + i) for i in range(procs)]))
    wall = time.perf_counter() - t0
    step_s = max(secs) / per
    out["serving_all_cores"] = {
        "sample": f"{procs} processes, each {per} steps of a 128^3 serving shot (sponge 20, line of receivers)",
        "cores": procs, "s_per_step_per_process": round(step_s, 4),
        "shots_per_s_128_extrapolated": round(procs / (step_s * 1250), 5),
        "note": "extrapolated to 1250 steps per shot; 128^3 is the smallest serving grid", "wall_s": round(wall, 1)}
    return out


_PROBE = None


def _probe_lib():
    """The hand-written stream kernels (libwave_probe.so, built with libwave)."""
    global _PROBE
    if _PROBE is None:
        import ctypes

        path = os.path.join(ROOT, "paper_2404_04441_amd", "libwave_probe.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} missing: build with python -m paper_2404_04441_amd.build")
        L = ctypes.CDLL(path)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.probe_stream_3r1w.argtypes = [vp, vp, vp, vp, sz, vp]
        L.probe_copy.argtypes = [vp, vp, sz, vp]
        L.probe_stream_16bit.argtypes = [vp, vp, vp, vp, vp, sz, ctypes.c_int, vp]
        _PROBE = L
    return _PROBE


def stream_ceiling(dev, n: int, reps: int = 20) -> dict:
    """What plain streams of the step's size reach on this GPU: hand-written
    HIP kernels over n float32 elements, with the step kernel's access
    policies (16-B lanes, nontemporal loads of the read-once arrays and
    nontemporal stores, XCD-remapped workgroups): d = a + b * c (3 reads + 1
    write, the float32 step's traffic shape) and a copy (1 read + 1 write)."""
    import torch

    n = n // 4 * 4
    lib = _probe_lib()
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    d = torch.empty_like(a)
    st = torch.cuda.current_stream(dev)
    out = {"kernel": "libwave_probe stream_3r1w / copy_1r1w", "elements": n}
    for name, fn, nbytes in (
            ("stream_3r1w", lambda: lib.probe_stream_3r1w(a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(), n,
                                                          st.cuda_stream), 16 * n),
            ("copy", lambda: lib.probe_copy(a.data_ptr(), d.data_ptr(), n, st.cuda_stream), 8 * n)):
        for _ in range(3):
            assert fn() == 0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_ms"] = round(ms, 4)
        out[f"{name}_gb_per_s"] = round(nbytes / ms / 1e6, 1)
    assert torch.equal(d[:4], a[:4])  # the copy ran
    del a, b, c, d
    torch.cuda.empty_cache()
    return out


def size_probe(n: int, steps: int = 30, tilings=()) -> dict:
    """One grid size N^3 (smooth random model, Dirichlet, a line of
    receivers): the HIP stream ceiling of that size, then the float32 step
    kernel in its tuned configuration; its algorithmic GB/s (16 B per point)
    against the ceiling.  Run under rocprofv3 counters, it gives the bytes
    each kernel moves per launch.  tilings: (variant, zchunk) pairs also
    timed with tuning off (20 steps, best of two runs each)."""
    import torch

    from paper_2404_04441_amd import Solver
    from synth import workload
    from synth.velocity import smooth_random_torch
    from synth.workloads import line_receivers

    dev = torch.device("cuda:0")
    W = workload("precision")
    out = {"grid": f"{n}^3", "ceiling": stream_ceiling(dev, n ** 3)}
    v = smooth_random_torch((n, n, n), seed=3, device=dev)
    rec = line_receivers(n, n // 2, 4)
    wav = torch.from_numpy(W.wavelet(steps)).to(dev)
    tr = torch.empty((steps, len(rec)), dtype=torch.float32, device=dev)
    s = Solver(v, W.h, W.dt, src=(n // 2, n // 2, n // 2), rec=rec)
    s.run(3, wav, tr)
    r = kernel_rate(s, steps, wav, tr, n ** 3, BYTES_PER_POINT["f32"])
    r["tiling"] = s.tiling()
    s.close()
    r["frac_of_stream_3r1w"] = round(r["gb_per_s"] / out["ceiling"]["stream_3r1w_gb_per_s"], 4)
    out["step_f32"] = r
    fixed = []
    for var, zc in tilings:
        s = Solver(v, W.h, W.dt, src=(n // 2, n // 2, n // 2), rec=rec, variant=var, zchunk=zc, tune=False)
        s.run(3, wav, tr)
        best = min((kernel_rate(s, 20, wav, tr, n ** 3, BYTES_PER_POINT["f32"]) for _ in range(2)),
                   key=lambda x: x["kernel_ms"])
        best["tiling"] = s.tiling()
        s.close()
        best["frac_of_stream_3r1w"] = round(best["gb_per_s"] / out["ceiling"]["stream_3r1w_gb_per_s"], 4)
        print(f"[bench] size probe {n}^3 variant {var} z-chunk {zc}: {best}", file=sys.stderr, flush=True)
        fixed.append(best)
    if fixed:
        out["fixed_tilings"] = fixed
    print(f"[bench] size probe {n}^3: {out}", file=sys.stderr, flush=True)
    return out


def copy_calibration(dev) -> None:
    """A plain device copy of known size (2 GiB read, 2 GiB written, three
    times): its FETCH_SIZE / WRITE_SIZE counters give the factor between
    counter readings and bytes moved."""
    import torch

    src = torch.ones(1 << 29, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x {src.numel() * 4} bytes read and written", file=sys.stderr, flush=True)
    del src, dst
    torch.cuda.empty_cache()


def stream16_ceiling(dev, n: int, reps: int = 20) -> dict:
    """The 16-bit storage step's traffic shape as a plain HIP stream over n
    nodes: A and V read at 2 B, m at 4 B (or 2 B as 16-bit codes), A' and V'
    written at 2 B, four nodes per lane, the step's cache policies and XCD
    remap.  As in a run of steps, A' goes to the other A buffer and becomes
    the next launch's input, and V is updated in place: a launch never reads
    the A it just read again (at 512^3 an A field is as large as the 256 MB
    last-level cache).  Rates in nodes per second, so each 16-bit form can be
    set against the stream of its own access shape."""
    import torch

    n = n // 4 * 4
    lib = _probe_lib()
    bufs = [torch.zeros(n, dtype=torch.int16, device=dev) for _ in range(2)]
    v = torch.zeros_like(bufs[0])
    m = torch.zeros(n, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream(dev)
    out = {"kernel": "libwave_probe stream_16bit", "nodes": n}
    for m16, key, bpp in ((0, "m_f32", 12), (1, "m_16bit", 10)):
        def fn(k):
            a, ao = bufs[k % 2], bufs[(k + 1) % 2]
            return lib.probe_stream_16bit(a.data_ptr(), v.data_ptr(), m.data_ptr(), ao.data_ptr(), v.data_ptr(), n,
                                          m16, st.cuda_stream)
        for k in range(3):
            assert fn(k) == 0
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for k in range(reps):
            fn(k + 1)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[key] = {"ms": round(ms, 4), "gpts_per_s": round(n / ms / 1e6, 2), "gb_per_s": round(bpp * n / ms / 1e6, 1)}
    del bufs, v, m
    torch.cuda.empty_cache()
    return out


def _frac_of_stream16(out: dict, ceiling: dict) -> None:
    """Each 16-bit form's rate against the stream of its own access shape."""
    for form, r in out.items():
        if isinstance(r, dict) and "gpts_per_s" in r and form != "f32":
            ref = ceiling["m_16bit" if form.endswith("_m16") else "m_f32"]["gpts_per_s"]
            r["frac_of_stream_16bit"] = round(r["gpts_per_s"] / ref, 4)


def kernel_rate(s, nt, wav, traces, npts, bpp, ref_bpp=None):
    """Average step-kernel time (events on the solver's stream) -> Gpts/s, GB/s
    and the fraction of 8 TB/s at bpp algorithmic bytes per point (and at
    ref_bpp, if given)."""
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.reset()
    e0.record(s.stream)
    s.step(nt, wav, traces)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nt
    out = {"kernel_ms": round(ms, 4), "gpts_per_s": round(npts / ms / 1e6, 2), "bytes_per_point": bpp,
           "gb_per_s": round(bpp * npts / ms / 1e6, 1), "roofline_frac": round(bpp * npts / ms / 1e6 / PEAK_HBM_GBS, 4)}
    if ref_bpp:
        out[f"roofline_frac_at_{ref_bpp}B"] = round(ref_bpp * npts / ms / 1e6 / PEAK_HBM_GBS, 4)
    return out


def _storage_kw(form):
    """Solver arguments of a storage form: "f16", "bf16_m16", ..."""
    fmt, _, m = form.partition("_")
    return {"storage": fmt, "model_bits": 16 if m == "m16" else 32}


def storage_forms_leg(W, vel_dev, nt: int) -> dict:
    """The 512^3 workload with 16-bit wavefield storage (float32 arithmetic)."""
    import torch

    from paper_2404_04441_amd import Solver

    out = {}
    wav = torch.from_numpy(W.wavelet(nt)).to(vel_dev.device)
    traces = torch.empty((nt, len(W.rec)), dtype=torch.float32, device=vel_dev.device)
    for fmt in ("f16", "bf16", "f16_m16", "bf16_m16"):
        s = Solver(vel_dev, W.h, W.dt, src=W.src, rec=W.rec, sponge_width=W.sponge_width,
                   sponge_alpha=W.sponge_alpha, **_storage_kw(fmt))
        s.run(20, wav, traces)
        out[fmt] = kernel_rate(s, nt, wav, traces, W.npts, BYTES_PER_POINT[fmt], SURVEY_16BIT_BYTES)
        out[fmt]["tiling"] = s.tiling()
        s.close()
    out["stream_16bit"] = stream16_ceiling(vel_dev.device, W.npts)
    _frac_of_stream16(out, out["stream_16bit"])
    return out


def cpml_leg(W, vel_dev, nt: int) -> dict:
    """The 512^3 workload with CPML layers of 20 nodes (the paper's boundary)
    instead of the sponge, float32: time per step of all kernels of a step.
    "fused": the automatic shape, whose step kernel applies the boundary terms
    (memory-variable pass + step).  "separate": variant 9 (same 4-node lanes,
    no fused kernel): memory-variable pass, plain step, boundary correction
    pass, receiver gather."""
    import torch

    from paper_2404_04441_amd import Solver

    wav = torch.from_numpy(W.wavelet(nt)).to(vel_dev.device)
    traces = torch.empty((nt, len(W.rec)), dtype=torch.float32, device=vel_dev.device)
    # algorithmic bytes of a CPML step: the plain step (16 B per point) plus, on
    # each axis' layer nodes, psi and zeta read and written once (16 B) and psi
    # read once more for its derivative (4 B)
    nz, ny, nx = W.shape
    wl = W.sponge_width
    layer_nodes = 2 * wl * (ny * nz + nx * nz + nx * ny)
    cpml_bytes = 16 * W.npts + 20 * layer_nodes
    out = {"layers": W.sponge_width, "reflection": 1e-3, "f0_hz": W.f0,
           "algorithmic_bytes_per_step": cpml_bytes,
           "note": "all kernels of a step; roofline_frac at 16 B/pt as the plain step, "
                   "roofline_frac_cpml at the CPML step's own algorithmic bytes"}
    for name, variant in (("fused", 0), ("separate", 9)):
        s = Solver(vel_dev, W.h, W.dt, src=W.src, rec=W.rec, cpml_width=W.sponge_width, cpml_f0=W.f0,
                   variant=variant)
        s.run(10, wav, traces)
        r = kernel_rate(s, nt, wav, traces, W.npts, BYTES_PER_POINT["f32"])
        tiling = s.tiling()
        s.close()
        out[name] = {"step_ms": r["kernel_ms"], "gpts_per_s": r["gpts_per_s"], "roofline_frac": r["roofline_frac"],
                     "roofline_frac_cpml": round(cpml_bytes / (r["kernel_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "tiling": tiling}
    return out


def precision_leg(nt: int = 500) -> dict:
    """The 1024^3 workload (smooth random model, 500 steps) in each storage type."""
    import torch

    from paper_2404_04441_amd import Solver
    from synth import workload
    from synth.velocity import smooth_random_torch

    W = workload("precision")
    dev = torch.device("cuda:0")
    vel = smooth_random_torch(W.shape, seed=3, device=dev)
    wav = torch.from_numpy(W.wavelet(nt)).to(dev)
    traces = torch.empty((nt, len(W.rec)), dtype=torch.float32, device=dev)
    out = {"workload": f"{W.name}, {nt} steps, Dirichlet, line of 1024 receivers"}
    for fmt in ("f32", "f16", "bf16", "f16_m16", "bf16_m16"):
        s = Solver(vel, W.h, W.dt, src=W.src, rec=W.rec, **_storage_kw(fmt))
        s.run(10, wav, traces)
        out[fmt] = kernel_rate(s, nt, wav, traces, W.npts, BYTES_PER_POINT[fmt],
                               None if fmt == "f32" else SURVEY_16BIT_BYTES)
        out[fmt]["tiling"] = s.tiling()
        s.close()
        print(f"[bench] precision 1024^3 {fmt}: {out[fmt]}", file=sys.stderr, flush=True)
    del vel
    torch.cuda.empty_cache()
    out["stream_ceiling"] = stream_ceiling(dev, W.npts)  # HIP streams of the 1024^3 size
    out["stream_16bit"] = stream16_ceiling(dev, W.npts)
    _frac_of_stream16(out, out["stream_16bit"])
    return out


# Seconds for 1024^3 x 1000 steps printed in the paper's Table "cuda-time"
# (NVIDIA GPUs, no thread-block clusters): context for the kernel study.
PAPER_CUDA_TIME_S = {
    "gmem": {"A100": 27.058, "GH200": 11.710},
    "smem": {"A100": 23.740, "GH200": 11.635},
    "st_reg_fixed": {"A100": 19.908, "GH200": 9.445},
    "st_semi": {"A100": 16.154, "GH200": 9.654},
}


def kernel_study_leg(nt: int = 20) -> dict:
    """The paper's kernel comparison rebuilt on one MI355X: its two 3D-blocking
    designs (gmem, smem), 2.5D streaming tile shapes and the 2.5D semi-stencil
    form (st_semi), each the whole fused
    float32 step, on the 1024^3 workload; the time for 1000 steps is 1000 x the
    average step-kernel time.  Then the grid-size sweep of the automatic shape
    (grid points per second against N, as in the paper's grid/s figure)."""
    import torch

    from paper_2404_04441_amd import Solver, variant_info
    from synth import workload
    from synth.velocity import smooth_random_torch
    from synth.workloads import line_receivers

    W = workload("precision")
    dev = torch.device("cuda:0")
    vel = smooth_random_torch(W.shape, seed=3, device=dev)
    wav = torch.from_numpy(W.wavelet(max(nt, 50))).to(dev)
    traces = torch.empty((max(nt, 50), len(W.rec)), dtype=torch.float32, device=dev)
    kernels = {"gmem (3D blocks 64x4x4, global memory)": 14, "smem (3D blocks 64x4x4 + halo in LDS)": 15,
               "2.5D 64x32, 1 node/lane, 3 planes in flight": 18, "2.5D 64x32, 1 node/lane, 1 plane in flight": 5,
               "2.5D 256x8, 4 nodes/lane": 12, "2.5D 128x32, 2 nodes/lane (automatic at 1024^2 planes)": 11,
               "2.5D semi-stencil 64x32, 1 node/lane": 16, "2.5D semi-stencil 256x8, 4 nodes/lane": 17}
    out = {"workload": f"{W.name}, float32, Dirichlet, {nt} timed steps per kernel",
           "paper_seconds_1000_steps": PAPER_CUDA_TIME_S}
    for name, v in kernels.items():
        s = Solver(vel, W.h, W.dt, src=W.src, rec=W.rec, variant=v)
        s.run(3, wav, traces)
        r = kernel_rate(s, nt, wav, traces, W.npts, BYTES_PER_POINT["f32"])
        r["variant"] = v
        r["shape"] = variant_info(v)
        r["seconds_1000_steps"] = round(r["kernel_ms"], 3)
        s.close()
        out[name] = r
        print(f"[bench] kernel study {name}: {r}", file=sys.stderr, flush=True)
    del vel
    torch.cuda.empty_cache()
    sweep, tuned, tilings = {}, {}, {}
    for n in (96, 128, 192, 256, 320, 384, 512, 640, 768, 896, 1024):
        v_n = smooth_random_torch((n, n, n), seed=3, device=dev)
        rec = line_receivers(n, n // 2, 4)
        tr = torch.empty((50, len(rec)), dtype=torch.float32, device=dev)
        steps = 50 if n <= 512 else nt
        tilings[str(n)] = {}
        for tune, dst, key in ((False, sweep, "fixed"), (True, tuned, "tuned")):
            s = Solver(v_n, W.h, W.dt, src=(n // 2, n // 2, n // 2), rec=rec, tune=tune)
            s.run(3, wav, tr)
            dst[str(n)] = kernel_rate(s, steps, wav, tr, n ** 3, BYTES_PER_POINT["f32"])["gpts_per_s"]
            tilings[str(n)][key] = s.tiling()
            s.close()
        del v_n
        torch.cuda.empty_cache()
    out["grid_sweep_gpts_per_s"] = sweep
    out["grid_sweep_tuned_gpts_per_s"] = tuned
    out["grid_sweep_tilings"] = tilings
    print(f"[bench] grid sweep: {sweep} tuned: {tuned}", file=sys.stderr, flush=True)
    return out


def temporal_blocking_leg() -> dict:
    """Two time steps per pass (time_block = 2) against one step per pass, on
    the cache-resident 256^3 grid (the fields fit the 256 MB last-level
    cache) and on the 512^3 grid: Gpts/s (points x time steps / time) and
    each form's algorithmic bytes per point-step (one step per pass: 16 B;
    a pass: A^n, A^{n-1}, m read and A^{n+1}, A^{n+2} written, 20 B for two
    steps, 10 B per step)."""
    import torch

    from paper_2404_04441_amd import Solver
    from synth import workload
    from synth.velocity import smooth_random_torch
    from synth.workloads import line_receivers

    W = workload("precision")
    dev = torch.device("cuda:0")
    out = {"note": "smooth random model, Dirichlet, centre source, line of receivers; kernel time only"}
    for n in (256, 512):
        v = smooth_random_torch((n, n, n), seed=3, device=dev)
        rec = line_receivers(n, n // 2, 4)
        steps = 200 if n <= 256 else 60
        wav = torch.from_numpy(W.wavelet(steps)).to(dev)
        tr = torch.empty((steps, len(rec)), dtype=torch.float32, device=dev)
        row = {}
        for name, kw, bpp in (("one_step_tuned", {}, 16), ("one_step_cached_policy", dict(cache_hint=1), 16),
                              ("two_steps_per_pass", dict(time_block=2), 10),
                              ("two_steps_per_pass_zchunk64", dict(time_block=2, zchunk=64), 10)):
            s = Solver(v, W.h, W.dt, src=(n // 2, n // 2, n // 2), rec=rec, **kw)
            s.run(4, wav, tr)
            r = kernel_rate(s, steps, wav, tr, n ** 3, bpp)
            r["tiling"] = s.tiling()
            s.close()
            row[name] = r
        out[f"{n}^3"] = row
        print(f"[bench] temporal blocking {n}^3: " + ", ".join(f"{k} {r['gpts_per_s']}" for k, r in row.items()),
              file=sys.stderr, flush=True)
        del v
        torch.cuda.empty_cache()
    return out


def gradient_leg(nt: int = 0, reps: int = 3) -> dict:
    """The 256^3 two-layer gradient workload (800 steps, sqrt(T) checkpoints):
    time of the velocity gradient against the time of the forward run
    (nt > 0: that many steps instead, for short profiled runs)."""
    import time as _t

    import numpy as np
    import torch

    from paper_2404_04441_amd import Solver
    from synth import workload
    from synth.velocity import smooth_along_z

    W = workload("gradient")
    nt = nt or W.nt
    dev = torch.device("cuda:0")
    v_true = W.velocity()
    v0 = smooth_along_z(v_true, 8.0)
    wav = torch.from_numpy(W.wavelet(nt)).to(dev)
    st = Solver(torch.from_numpy(v_true).to(dev), W.h, W.dt, src=W.src, rec=W.rec)
    d_obs = st.run(nt, wav).clone()
    st.close()
    s = Solver(torch.from_numpy(v0).to(dev), W.h, W.dt, src=W.src, rec=W.rec, adjoint=True, nt_max=nt)
    tr = s.run(nt, wav)
    resid = (tr - d_obs).contiguous()
    grad = s.adjoint(nt, wav, resid)  # warm-up
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    for _ in range(reps):
        s.run(nt, wav, tr)
    torch.cuda.synchronize()
    t_fwd = (_t.perf_counter() - t0) / reps
    t0 = _t.perf_counter()
    for _ in range(reps):
        s.adjoint(nt, wav, resid, grad)
    torch.cuda.synchronize()
    t_grad = (_t.perf_counter() - t0) / reps
    misfit = 0.5 * float((resid.double() ** 2).sum())
    s.close()
    # per gradient point-step: forward with checkpoints 16 + recomputation 16 +
    # storing it 4 + adjoint step 16 + reading the forward field 4 + the
    # imaging accumulator read and written 8
    bytes_per_pt_step = 64
    return {"workload": f"{W.name}, {nt} steps, two-layer model, smoothed start, 256x256 receivers, "
                        f"checkpoint every {int(np.ceil(np.sqrt(nt)))} steps",
            "forward_s": round(t_fwd, 4), "gradient_s": round(t_grad, 4), "ratio": round(t_grad / t_fwd, 3),
            "gradient_gpts_per_s": round(W.npts * nt / t_grad / 1e9, 2),
            "gradient_gb_per_s": round(bytes_per_pt_step * W.npts * nt / t_grad / 1e9, 1),
            "bytes_per_gradient_point_step": bytes_per_pt_step,
            "roofline_frac": round(bytes_per_pt_step * W.npts * nt / t_grad / 1e9 / PEAK_HBM_GBS, 4),
            "misfit": misfit, "grad_finite": bool(torch.isfinite(grad).all().item())}


def serving_leg(count: int, lanes: int = 0, slots: int = 8) -> dict:
    """Serve the seeded Poisson stream of forward-shot requests (512 at 20/s;
    grids 128^3 .. 384^3, 500..2000 steps, f32 or f16 storage).  Each grid
    class is tuned once before the stream starts; admission is bounded by the
    device memory free at that point (less a 4 GiB reserve)."""
    import time as _t

    import torch

    from paper_2404_04441_amd.serve import GpuBackend, ShotServer, requests_from_workload, summarize

    reqs = requests_from_workload(count)
    backend = GpuBackend(graph_steps=20, lanes=lanes)
    t0 = _t.perf_counter()
    tuned = backend.pretune(reqs)
    t_tune = _t.perf_counter() - t0
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    budget = max(free - (4 << 30), 1 << 30)
    print(f"[bench] serving {count} shot requests; tuned {len(tuned)} classes in {t_tune:.1f} s; "
          f"admission budget {budget / 2**30:.1f} GiB of {total / 2**30:.1f}", file=sys.stderr, flush=True)
    server = ShotServer(backend, budget_bytes=budget, max_slots=slots, chunk_steps=200)
    res = server.run(reqs)
    out = summarize(res, reqs, server.elapsed)
    out["max_concurrent"] = server.max_concurrent
    out["slots"] = slots
    out["lanes"] = lanes
    out["budget_gib"] = round(budget / 2**30, 1)
    out["pretune_s"] = round(t_tune, 2)
    out["workload"] = (f"{count} Poisson shot requests at 20/s (seed 5): grids 128^3, 256x192x128, 256^3, 384^3; "
                       f"500..2000 steps; f32 or f16 storage; 20-node sponge; line of receivers")
    print(f"[bench] serving done: {out}", file=sys.stderr, flush=True)
    return out


def small_shot_probe(nt: int = 2000) -> dict:
    """One 128^3 serving shot alone (f32, sponge, line of receivers), stepped
    by graph replay as the server does: wall time per step.  Compared with
    the step kernel's own duration (rocprofv3 kernel trace of this leg) it
    shows how much of a small shot's time is launch overhead."""
    import torch

    from paper_2404_04441_amd import Solver
    from paper_2404_04441_amd.serve import requests_from_workload

    req = next(r for r in requests_from_workload(512) if r.shape == (128, 128, 128) and r.storage == "f32")
    dev = torch.device("cuda:0")
    vel = torch.from_numpy(np.ascontiguousarray(req.velocity, dtype=np.float32)).to(dev)
    vel = vel.view(-1, 1, 1).expand(req.shape).contiguous()
    from synth.wavelet import ricker
    wav = torch.from_numpy(ricker(nt, req.dt, req.f0, req.t0)).to(dev)
    tr = torch.empty((nt, len(req.rec)), dtype=torch.float32, device=dev)
    out = {"grid": "128^3 f32, sponge 20, line of 128 receivers", "steps": nt}
    for graph in (0, 20):
        s = Solver(vel, req.h, req.dt, src=req.src, rec=req.rec, sponge_width=req.sponge_width,
                   sponge_alpha=req.sponge_alpha, graph_steps=graph)
        s.run(nt, wav, tr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            s.run(nt, wav, tr)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 3 / nt * 1e3
        out[f"ms_per_step_graph{graph}"] = round(ms, 5)
        out["tiling"] = s.tiling()
        s.close()
    print(f"[bench] small-shot probe: {out}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--tune", action="store_true",
                    help="create-time tuning (shape, z-chunk, cache policy; outside the timed region) instead of "
                         "the fixed rule, whose 512^3 choice tuning also finds; the fixed rule keeps counter runs "
                         "on one kernel configuration")
    ap.add_argument("--nt", type=int, default=0, help="time steps per shot (default: the workload's 1000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the 16-bit, CPML, 1024^3, kernel-study and gradient measurements")
    ap.add_argument("--serving", type=int, default=512,
                    help="requests of the Poisson shot stream to serve after the throughput run (0: skip)")
    ap.add_argument("--serving-lanes", type=int, default=0,
                    help="serving: 0 = shots' kernels overlap freely; k = at most k kernels in flight")
    ap.add_argument("--serving-slots", type=int, default=8, help="serving: shots admitted at once")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg and the small-shot probe and print their JSON")
    ap.add_argument("--study-only", action="store_true",
                    help="run only the 1024^3 kernel study (3D gmem/smem vs 2.5D shapes) and print its JSON")
    ap.add_argument("--cpml-only", action="store_true",
                    help="run only the 512^3 CPML leg (fused and unfused shapes) and print its JSON")
    ap.add_argument("--forms-only", action="store_true",
                    help="run only the 512^3 16-bit storage forms (and their stream probe) and print JSON")
    ap.add_argument("--precision-only", action="store_true",
                    help="run only the 1024^3 storage forms (float32, 16-bit, 16-bit with 16-bit m) and print JSON")
    ap.add_argument("--gradient-only", action="store_true",
                    help="run only the 256^3 x 800 gradient leg and print its JSON")
    ap.add_argument("--size-probe", type=int, default=0,
                    help="run only the N^3 size probe (HIP stream ceiling + tuned float32 step) and print its JSON")
    ap.add_argument("--probe-tilings", default="",
                    help="with --size-probe: also time these fixed tilings, 'variant:zchunk,...' (tuning off)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (one shot per GPU).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2404_04441_amd import Solver
    from synth import workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.study_only:
        print(json.dumps({"kernel_study_1024": kernel_study_leg()}), flush=True)
        return
    if args.size_probe:
        if args.copy_calibration:
            copy_calibration(torch.device("cuda:0"))
        pairs = [tuple(int(x) for x in t.split(":")) for t in args.probe_tilings.split(",") if t]
        print(json.dumps({"size_probe": size_probe(args.size_probe, tilings=pairs)}), flush=True)
        return
    if args.precision_only:
        if args.copy_calibration:
            copy_calibration(torch.device("cuda:0"))
        print(json.dumps({"precision_1024": precision_leg(args.nt or 500)}), flush=True)
        return
    if args.gradient_only:
        if args.copy_calibration:
            copy_calibration(torch.device("cuda:0"))
        print(json.dumps({"gradient_256": gradient_leg(args.nt, args.steps if args.nt else 3)}), flush=True)
        return
    if args.serving_only:
        out = {"small_shot_probe": small_shot_probe()}
        if args.serving > 0:
            out["serving"] = serving_leg(args.serving, args.serving_lanes, args.serving_slots)
        print(json.dumps(out), flush=True)
        return
    dev = torch.device("cuda:0")
    W = workload("large")
    if args.cpml_only:
        if args.copy_calibration:
            copy_calibration(dev)
        v_dev = torch.from_numpy(W.velocity()).to(dev)
        print(json.dumps({"cpml_512": cpml_leg(W, v_dev, min(args.nt or W.nt, 200))}), flush=True)
        return
    if args.forms_only:
        if args.copy_calibration:
            copy_calibration(dev)
        v_dev = torch.from_numpy(W.velocity()).to(dev)
        print(json.dumps({"forms_512": storage_forms_leg(W, v_dev, min(args.nt or W.nt, 200))}), flush=True)
        return
    nt = args.nt or W.nt
    print(f"[bench] building {W.name} inputs", file=sys.stderr, flush=True)
    vel = W.velocity()
    wav = torch.from_numpy(W.wavelet(nt)).to(dev)
    s = Solver(torch.from_numpy(vel).to(dev), W.h, W.dt, src=W.src, rec=W.rec, sponge_width=W.sponge_width,
               sponge_alpha=W.sponge_alpha, storage=args.storage, variant=args.variant, zchunk=args.zchunk,
               tune=args.tune)
    traces = torch.empty((nt, len(W.rec)), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        s.run(nt, wav, traces)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.run(nt, wav, traces)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = W.npts * nt * args.steps / wall / 1e9
    print(f"[bench] timed {args.steps} shots: {ms_per_step:.1f} ms/shot", file=sys.stderr, flush=True)

    # step-kernel duration: events on the solver's own stream around step kernels only
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.reset()
    e0.record(s.stream)
    s.step(nt, wav, traces)
    e1.record(s.stream)
    torch.cuda.synchronize()
    kernel_ms = e0.elapsed_time(e1) / nt
    bpp = BYTES_PER_POINT[args.storage]
    achieved = bpp * W.npts / (kernel_ms * 1e-3) / 1e9
    flags = s.sync_status()
    tiling = s.tiling()
    s.close()

    if args.copy_calibration:
        copy_calibration(dev)
    ceiling = stream_ceiling(dev, W.npts)

    out = {
        "metric": "stencil Gpts/s & % HBM roofline (1 GPU); shots/s with p50/p99 latency",
        "value": round(value, 2),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"{args.storage} storage, f32 arithmetic",
        "data": "synthetic",
        "config": {"workload": f"{W.name} FP32 fused forward shot: 8th-order star stencil, leapfrog, "
                               f"20-node sponge, Ricker source at (256,256,10), 512x512 receiver plane z=0",
                   "grid": list(W.shape[::-1]), "time_steps": nt, "storage": args.storage,
                   "variant": args.variant, "zchunk": args.zchunk, "tuned": bool(args.tune), "tiling": tiling},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(args.storage, tiling),
                     "kernel": "step_kernel", "kernel_ms": round(kernel_ms, 4),
                     "algorithmic_bytes_per_launch": bpp * W.npts},
        "nonfinite": bool(flags),
        "stream_ceiling": ceiling,
    }
    if not args.no_forms:
        v_dev = torch.from_numpy(vel).to(dev)
        out["forms_512"] = storage_forms_leg(W, v_dev, min(nt, 200))
        out["cpml_512"] = cpml_leg(W, v_dev, min(nt, 200))
        print(f"[bench] cpml: {out['cpml_512']}", file=sys.stderr, flush=True)
        del v_dev
        out["precision_1024"] = precision_leg()
        out["kernel_study_1024"] = kernel_study_leg()
        out["temporal_blocking"] = temporal_blocking_leg()
        out["gradient_256"] = gradient_leg()
        print(f"[bench] gradient: {out['gradient_256']}", file=sys.stderr, flush=True)
    if args.serving > 0:
        out["small_shot_probe"] = small_shot_probe()
        out["serving"] = serving_leg(args.serving, args.serving_lanes, args.serving_slots)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, vel)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
