"""Python front of libwave: torch supplies device memory and the stream.

Every step of the computation runs in libwave's HIP kernels; this module only
allocates the workspace, marshals pointers and checks status codes.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")
    return t


class Solver:
    """One shot of the fused 8th-order acoustic solver on one GPU.

    vel      : float32 [nz, ny, nx] velocity on the GPU (m/s)
    h        : grid spacing, scalar or (dx, dy, dz)
    dt       : time step (s)
    src      : (ix, iy, iz) or None
    rec      : int array [nrec, 3] of (ix, iy, iz) or None
    storage  : "f32", "f16" or "bf16" wavefield storage
    adjoint  : reserve the adjoint workspace for runs up to ``nt_max`` steps
    variant, zchunk, graph_steps : kernel tiling / replay options
    tune : time the candidate tile shapes at create and keep the fastest (cached per grid shape; default on,
           False = the fixed rule)
    cpml_width, cpml_reflection, cpml_f0 : CPML absorbing layers (float32 forward; sponge_width must be 0)
    cache_hint : 1 = keep the fields read or written once cacheable (grids that fit the last-level
                 cache); 0 = nontemporal (tune also times the cacheable policy)
    model_bits : 32 (default) = m = (v dt)^2 in float32; 16 = a 16-bit affine code of m (16-bit
                 storage only; relative error in m <= (m_max / m_min - 1) / 131070, 10 B per node-step)
    time_block : 2 = two time steps per pass over the grid (float32 forward; same bits), 0 = one
    """

    def __init__(self, vel: torch.Tensor, h, dt: float, src=None, rec=None, sponge_width: int = 0,
                 sponge_alpha: float = 0.015, storage: str = "f32", adjoint: bool = False, nt_max: int = 0,
                 ckpt_interval: int = 0, variant: int = 0, zchunk: int = 0, graph_steps: int = 0, tune: bool = True,
                 cpml_width: int = 0, cpml_reflection: float = 1e-3, cpml_f0: float = 0.0, cache_hint: int = 0,
                 model_bits: int = 32, time_block: int = 0, stream=None):
        lib = L.lib()
        _dev_f32(vel, "vel")
        nz, ny, nx = vel.shape
        hx, hy, hz = (h, h, h) if np.isscalar(h) else h
        p = L.WaveParams()
        lib.wave_params_init(ctypes.byref(p))
        p.nx, p.ny, p.nz = nx, ny, nz
        p.dx, p.dy, p.dz, p.dt = float(hx), float(hy), float(hz), float(dt)
        p.sponge_width, p.sponge_alpha = int(sponge_width), float(sponge_alpha)
        p.storage = L.STORAGE[storage]
        if src is None:
            p.src[0], p.src[1], p.src[2] = -1, 0, 0
        else:
            p.src[0], p.src[1], p.src[2] = (int(c) for c in src)
        self._rec = np.ascontiguousarray(np.zeros((0, 3)) if rec is None else rec, dtype=np.int32).reshape(-1, 3)
        p.nrec = len(self._rec)
        p.rec = self._rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if p.nrec else None
        p.adjoint, p.nt_max, p.ckpt_interval = int(bool(adjoint)), int(nt_max), int(ckpt_interval)
        p.variant, p.zchunk, p.graph_steps = int(variant), int(zchunk), int(graph_steps)
        p.tune = 1 if tune else 0
        p.cpml_width, p.cpml_reflection, p.cpml_f0 = int(cpml_width), float(cpml_reflection), float(cpml_f0)
        p.cache_hint = int(cache_hint)
        p.model_bits = int(model_bits)
        p.time_block = int(time_block)
        nbytes = ctypes.c_size_t()
        L.check(lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(nbytes)), "wave_workspace_bytes")
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=vel.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(vel.device)
        self.device = vel.device
        self.shape = (nz, ny, nx)
        self.nrec = p.nrec
        self.has_source = src is not None
        self.storage = storage
        self._params = p
        handle = ctypes.c_void_p()
        with torch.cuda.device(vel.device):
            L.check(lib.wave_create(ctypes.byref(p), _ptr(vel), self._ws_ptr, self.workspace_bytes,
                                    self.stream.cuda_stream, ctypes.byref(handle)), "wave_create")
        self._h = handle

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().wave_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers
    def _traces(self, rows: int, traces):
        if self.nrec == 0:
            return None
        if traces is None:
            traces = torch.empty((rows, self.nrec), dtype=torch.float32, device=self.device)
        _dev_f32(traces, "traces")
        if traces.numel() < rows * self.nrec:
            raise ValueError("traces too small")
        return traces

    def _wavelet(self, wavelet, rows: int):
        if not self.has_source:
            return None
        _dev_f32(wavelet, "wavelet")
        if wavelet.numel() < rows:
            raise ValueError("wavelet too short")
        return wavelet

    # -- API
    def reset(self):
        L.check(L.lib().wave_reset(self._h), "wave_reset")

    def run(self, nt: int, wavelet=None, traces=None):
        """Reset and advance nt steps; returns traces [nt, nrec] (or None)."""
        wavelet = self._wavelet(wavelet, nt)
        traces = self._traces(nt, traces)
        L.check(L.lib().wave_run(self._h, int(nt), _ptr(wavelet), _ptr(traces)), "wave_run")
        return traces

    def step(self, nsteps: int, wavelet=None, traces=None):
        """Advance nsteps from the current n; wavelet/traces cover the whole
        run (absolute rows)."""
        n = self.time_index()
        wavelet = self._wavelet(wavelet, n + nsteps)
        traces = self._traces(n + nsteps, traces)
        L.check(L.lib().wave_step(self._h, int(nsteps), _ptr(wavelet), _ptr(traces)), "wave_step")
        return traces

    def adjoint(self, nt: int, wavelet, resid, grad=None):
        """dJ/dv for J with dJ/dtraces = resid [nt, nrec]."""
        wavelet = self._wavelet(wavelet, nt)
        if self.nrec:
            _dev_f32(resid, "resid")
            if resid.numel() < nt * self.nrec:
                raise ValueError("resid too small")
        if grad is None:
            grad = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _dev_f32(grad, "grad")
        L.check(L.lib().wave_adjoint(self._h, int(nt), _ptr(wavelet), _ptr(resid) if self.nrec else 0,
                                     _ptr(grad)), "wave_adjoint")
        return grad

    def read_field(self, which: int = 0, out=None):
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _dev_f32(out, "out")
        L.check(L.lib().wave_read_field(self._h, int(which), _ptr(out)), "wave_read_field")
        return out

    def write_field(self, which: int, field: torch.Tensor):
        """Set a stored time level from a float32 [nz, ny, nx] device tensor:
        A^n (which = 0) and, with float32 storage, the stored A^{n-1} (which = 1)
        or, with 16-bit storage, V^n (which = 2), encoded at the step rule's
        scale for its maximum."""
        _dev_f32(field, "field")
        if tuple(field.shape) != self.shape:
            raise ValueError(f"field must have shape {self.shape}")
        L.check(L.lib().wave_write_field(self._h, int(which), _ptr(field)), "wave_write_field")

    def save_state(self, out=None) -> torch.Tensor:
        """Snapshot of the shot (device bytes) that ``load_state`` resumes from."""
        n = ctypes.c_size_t()
        L.check(L.lib().wave_state_bytes(self._h, ctypes.byref(n)), "wave_state_bytes")
        if out is None:
            out = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        if out.numel() * out.element_size() < n.value or not out.is_cuda:
            raise ValueError(f"snapshot buffer must be a device tensor of at least {n.value} bytes")
        L.check(L.lib().wave_save_state(self._h, ctypes.c_void_p(out.data_ptr())), "wave_save_state")
        return out

    def load_state(self, snapshot: torch.Tensor):
        """Resume from a snapshot taken from a solver with the same parameters."""
        L.check(L.lib().wave_load_state(self._h, ctypes.c_void_p(snapshot.data_ptr())), "wave_load_state")

    def time_index(self) -> int:
        n = ctypes.c_int32()
        L.check(L.lib().wave_time_index(self._h, ctypes.byref(n)), "wave_time_index")
        return n.value

    def tiling(self) -> dict:
        """The forward configuration in use: variant, zchunk, cache_hint (pass
        them back to the constructor to reproduce a tuned choice)."""
        out = (ctypes.c_int32 * 3)()
        L.check(L.lib().wave_tiling(self._h, out), "wave_tiling")
        return {"variant": int(out[0]), "zchunk": int(out[1]), "cache_hint": int(out[2])}

    def sync_status(self) -> int:
        f = ctypes.c_uint32()
        L.check(L.lib().wave_sync_status(self._h, ctypes.byref(f)), "wave_sync_status")
        return f.value


def variant_count() -> int:
    return int(L.lib().wave_variant_count())


def variant_info(variant: int) -> dict:
    """Shape of a kernel variant: family (0 = 2.5D streaming, 1 = 3D gmem,
    2 = 3D smem), by, ry, pd, vec."""
    info = (ctypes.c_int32 * 5)()
    L.check(L.lib().wave_variant_info(int(variant), info), "wave_variant_info")
    return dict(zip(("family", "by", "ry", "pd", "vec"), (int(v) for v in info)))
