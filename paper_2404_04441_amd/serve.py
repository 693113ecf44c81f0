"""Continuous-batching server for independent forward shots.

Requests (one forward solve each: grid, step count, storage type, velocity)
arrive over time.  The scheduler admits a waiting request as soon as a slot
is free and its device footprint fits the memory budget, so shots that arrive
while others run join immediately; every admitted shot runs on its own
stream, advanced in chunks of captured-graph step replays, and is retired
(its workspace returned) when its last chunk's event completes.

The scheduler is backend-agnostic: ``GpuBackend`` drives libwave through
``Solver``; tests substitute a host-only backend to exercise admission,
ordering and failure handling without a GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

from . import _lib as L


@dataclass
class ShotRequest:
    id: int
    arrival: float          # seconds after the server starts
    shape: tuple            # (nz, ny, nx)
    nt: int
    storage: str            # "f32" | "f16" | "bf16"
    h: float
    dt: float
    src: tuple              # (ix, iy, iz)
    rec: np.ndarray         # int [nrec, 3]
    f0: float = 15.0
    t0: Optional[float] = None
    sponge_width: int = 20
    sponge_alpha: float = 0.015
    velocity: Any = None    # np.ndarray [nz, ny, nx] or a 1D z profile (layered model)

    @property
    def npts(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz


@dataclass
class ShotResult:
    id: int
    status: str             # "done" | "failed" | "rejected"
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    traces: Any = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class _Active:
    req: ShotRequest
    handle: Any
    footprint: int
    done_steps: int = 0
    admitted: float = 0.0
    inflight: List[Any] = field(default_factory=list)   # backend chunk tokens
    cancelled: bool = False


class ShotServer:
    """Admit, overlap and retire shots.

    budget_bytes : device memory the shots' footprints may occupy together
    max_slots    : shots running at once
    chunk_steps  : time steps per enqueued chunk (a few graph replays)
    depth        : chunks kept queued per shot, so the device never idles on the host
    """

    def __init__(self, backend, budget_bytes: int, max_slots: int = 8, chunk_steps: int = 200, depth: int = 2):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk_steps)
        self.depth = int(depth)

    def run(self, requests: List[ShotRequest], clock=time.perf_counter, sleep=time.sleep,
            cancel: Optional[set] = None) -> Dict[int, ShotResult]:
        cancel = cancel if cancel is not None else set()  # the caller may add ids while running
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        waiting: List[ShotRequest] = []
        active: List[_Active] = []
        results: Dict[int, ShotResult] = {}
        used = 0
        self.max_concurrent = 0
        t_start = clock()
        while pending or waiting or active:
            now = clock() - t_start
            while pending and pending[0].arrival <= now:
                waiting.append(pending.pop(0))
            # admission: FIFO, by slot and by footprint
            while waiting and len(active) < self.max_slots:
                req = waiting[0]
                if req.id in cancel:
                    waiting.pop(0)
                    results[req.id] = ShotResult(req.id, "failed", req.arrival, error="cancelled")
                    continue
                try:
                    need = int(self.backend.footprint(req))
                except Exception as e:  # invalid request: reject without blocking the queue
                    waiting.pop(0)
                    results[req.id] = ShotResult(req.id, "rejected", req.arrival, error=str(e))
                    continue
                if need > self.budget:
                    waiting.pop(0)
                    results[req.id] = ShotResult(req.id, "rejected", req.arrival,
                                                 error=f"footprint {need} exceeds the budget {self.budget}")
                    continue
                if used + need > self.budget:
                    break  # wait for memory to free up; keep arrival order
                waiting.pop(0)
                try:
                    handle = self.backend.start(req)
                except Exception as e:
                    results[req.id] = ShotResult(req.id, "failed", req.arrival, admitted=now, finished=now,
                                                 error=str(e))
                    continue
                used += need
                active.append(_Active(req, handle, need, admitted=clock() - t_start))
            self.max_concurrent = max(self.max_concurrent, len(active))
            # keep every active shot `depth` chunks ahead; retire finished ones
            progressed = False
            for a in list(active):
                a.inflight = [c for c in a.inflight if not self.backend.chunk_done(a.handle, c)]
                if a.req.id in cancel and a.done_steps < a.req.nt:
                    a.done_steps = a.req.nt  # stop enqueueing; retire once the queued chunks drain
                    a.cancelled = True
                while len(a.inflight) < self.depth and a.done_steps < a.req.nt:
                    n = min(self.chunk, a.req.nt - a.done_steps)
                    a.inflight.append(self.backend.advance(a.handle, n))
                    a.done_steps += n
                    progressed = True
                if a.done_steps >= a.req.nt and not a.inflight:
                    t = clock() - t_start
                    if a.cancelled:
                        results[a.req.id] = ShotResult(a.req.id, "failed", a.req.arrival, a.admitted, t,
                                                       error="cancelled")
                    else:
                        try:
                            tr = self.backend.result(a.handle)
                            results[a.req.id] = ShotResult(a.req.id, "done", a.req.arrival, a.admitted, t, tr)
                        except Exception as e:
                            results[a.req.id] = ShotResult(a.req.id, "failed", a.req.arrival, a.admitted, t,
                                                           error=str(e))
                    self.backend.release(a.handle)
                    used -= a.footprint
                    active.remove(a)
                    progressed = True
            if not progressed:
                nxt = pending[0].arrival - (clock() - t_start) if pending else None
                sleep(min(2e-4, nxt) if nxt is not None and nxt > 0 else 2e-4)
        self.elapsed = clock() - t_start
        return results


def summarize(results: Dict[int, ShotResult], requests: List[ShotRequest], elapsed: float) -> dict:
    done = [r for r in results.values() if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    by_id = {q.id: q for q in requests}
    served_pts = sum(by_id[r.id].npts * by_id[r.id].nt for r in done)
    offered = sum(q.npts * q.nt for q in requests)
    span = max(q.arrival for q in requests) if requests else 0.0
    return {
        "requests": len(requests),
        "done": len(done),
        "failed": sum(r.status == "failed" for r in results.values()),
        "rejected": sum(r.status == "rejected" for r in results.values()),
        "elapsed_s": round(elapsed, 3),
        "shots_per_s": round(len(done) / elapsed, 3) if elapsed > 0 else None,
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4) if lat.size else None,
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4) if lat.size else None,
        "mean_latency_s": round(float(lat.mean()), 4) if lat.size else None,
        "served_gpts_per_s": round(served_pts / elapsed / 1e9, 2) if elapsed > 0 else None,
        "offered_gpts_per_s": round(offered / span / 1e9, 2) if span > 0 else None,
    }


class GpuBackend:
    """Runs shots through libwave (one Solver per shot).

    Every shot runs on a stream of its own.  lanes = 0: the shots' chunks
    are independent, so their kernels may overlap on the device.  lanes =
    k > 0: the admitted shots are assigned round-robin to k lanes, and each
    chunk waits (an event) for the chunk queued before it on its lane, so at
    most k kernels overlap while every admitted shot keeps progressing chunk
    by chunk.  Overlapping kernels of several grids share the caches and
    the CUs less efficiently than one kernel at a time (measured: the GPU
    busy 98.7% of a serving run with 1.72 kernels in flight on average,
    yet below the shots' one-at-a-time rates)."""

    def __init__(self, device=None, graph_steps: int = 20, variant: int = 0, tune: bool = True, lanes: int = 0):
        import torch

        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.graph_steps = graph_steps
        self.variant = variant
        self.tune = tune  # time the tile shapes once per grid shape (libwave caches the choice)
        self.lanes = [None] * int(lanes)  # last chunk event queued on each lane
        self._next = 0

    def pretune(self, requests: List[ShotRequest]) -> dict:
        """Create (and close) one solver per distinct (grid, storage, sponge)
        class of ``requests`` before serving, so that libwave's create-time
        tuning of each class runs on an idle device instead of under the
        contention of running shots (the choice is cached per grid shape for
        the process).  Returns {class: seconds}."""
        import time

        torch = self.torch
        from synth.wavelet import ricker  # noqa: F401  (keeps the import cost out of the timed stream)

        from .solver import Solver

        if not (self.tune and self.variant == 0):
            return {}
        seen, out = set(), {}
        for req in requests:
            key = (tuple(req.shape), req.storage, req.sponge_width)
            if key in seen:
                continue
            seen.add(key)
            t0 = time.perf_counter()
            stream = torch.cuda.Stream(device=self.device)
            with torch.cuda.stream(stream):
                v = np.ascontiguousarray(req.velocity, dtype=np.float32)
                vel = torch.from_numpy(v).to(self.device)
                if v.ndim == 1:
                    vel = vel.view(-1, 1, 1).expand(req.shape).contiguous()
                s = Solver(vel, req.h, req.dt, src=req.src, rec=req.rec, sponge_width=req.sponge_width,
                           sponge_alpha=req.sponge_alpha, storage=req.storage, graph_steps=self.graph_steps,
                           tune=True, stream=stream)
                s.close()
            stream.synchronize()
            out["%dx%dx%d %s" % (req.shape[2], req.shape[1], req.shape[0], req.storage)] = round(
                time.perf_counter() - t0, 3)
        return out

    def footprint(self, req: ShotRequest) -> int:
        import ctypes

        lib = L.lib()
        p = L.WaveParams()
        lib.wave_params_init(ctypes.byref(p))
        nz, ny, nx = req.shape
        p.nx, p.ny, p.nz = nx, ny, nz
        p.dx = p.dy = p.dz = float(req.h)
        p.dt = float(req.dt)
        p.sponge_width, p.sponge_alpha = req.sponge_width, req.sponge_alpha
        p.storage = L.STORAGE[req.storage]
        p.src[0], p.src[1], p.src[2] = req.src
        rec = np.ascontiguousarray(req.rec, dtype=np.int32)
        p.nrec = len(rec)
        p.rec = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if len(rec) else None
        b = ctypes.c_size_t()
        L.check(lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)), "wave_workspace_bytes")
        # workspace + traces + wavelet + the velocity staged for create
        return b.value + 256 + 4 * req.nt * len(rec) + 4 * req.nt + 4 * req.npts

    def start(self, req: ShotRequest):
        torch = self.torch
        from synth.wavelet import ricker

        from .solver import Solver

        stream = torch.cuda.Stream(device=self.device)
        lane = None
        if self.lanes:
            lane = self._next % len(self.lanes)
            self._next += 1
        with torch.cuda.stream(stream):
            v = req.velocity
            if v.ndim == 1:  # layered model: expand the z profile on the device
                vel = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(self.device, non_blocking=False)
                vel = vel.view(-1, 1, 1).expand(req.shape).contiguous()
            else:
                vel = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(self.device)
            wav = torch.from_numpy(ricker(req.nt, req.dt, req.f0, req.t0)).to(self.device)
            traces = torch.empty((req.nt, len(req.rec)), dtype=torch.float32, device=self.device)
            s = Solver(vel, req.h, req.dt, src=req.src, rec=req.rec, sponge_width=req.sponge_width,
                       sponge_alpha=req.sponge_alpha, storage=req.storage, variant=self.variant,
                       graph_steps=self.graph_steps, tune=self.tune and self.variant == 0, stream=stream)
            del vel  # m now lives in the workspace
        return {"solver": s, "stream": stream, "wav": wav, "traces": traces, "lane": lane}

    def advance(self, h, nsteps: int):
        torch = self.torch
        s = h["solver"]
        lane = h["lane"]
        if lane is not None and self.lanes[lane] is not None:
            h["stream"].wait_event(self.lanes[lane])
        L.check(L.lib().wave_step(s._h, int(nsteps), int(h["wav"].data_ptr()), int(h["traces"].data_ptr())),
                "wave_step")
        ev = torch.cuda.Event()
        ev.record(h["stream"])
        if lane is not None:
            self.lanes[lane] = ev
        return ev

    def chunk_done(self, h, ev) -> bool:
        return ev.query()

    def result(self, h):
        h["stream"].synchronize()
        if h["solver"].sync_status():
            raise RuntimeError("non-finite wavefield")
        return h["traces"]

    def release(self, h):
        h["stream"].synchronize()
        h["solver"].close()
        h.clear()


def requests_from_workload(count: int = 512, rate: float = 20.0, seed: int = 5) -> List[ShotRequest]:
    """The Poisson stream of forward shots with per-request layered velocity
    models (z profiles, expanded on the device)."""
    from synth.velocity import layered_profile
    from synth.workloads import serving_requests

    out = []
    for d in serving_requests(count, rate, seed):
        out.append(ShotRequest(id=d["id"], arrival=d["arrival"], shape=d["shape"], nt=d["nt"],
                               storage=d["storage"], h=d["h"], dt=d["dt"], src=d["src"], rec=d["rec"],
                               f0=d["f0"], t0=d["t0"], sponge_width=d["sponge_width"],
                               sponge_alpha=d["sponge_alpha"],
                               velocity=layered_profile(d["shape"][0], d["velocity_seed"])))
    return out
