"""The synthetic workloads: grids, geometry, time step and source.

Arrays are indexed ``[z, y, x]``; receiver and source coordinates are given
as ``(ix, iy, iz)`` node triples (0-based).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import velocity as V
from .wavelet import ricker

# v_max * dt / h used by every workload: half of the 3D stability bound of the
# 8th-order/leapfrog scheme, 2 / sqrt(3 * 2048/315) = 0.452855...
COURANT = 0.22642776165920997


def line_receivers(nx: int, iy: int, iz: int) -> np.ndarray:
    """Receivers at x = 0..nx-1 on the line (y=iy, z=iz), in x order."""
    r = np.zeros((nx, 3), dtype=np.int32)
    r[:, 0] = np.arange(nx)
    r[:, 1] = iy
    r[:, 2] = iz
    return r


def plane_receivers(nx: int, ny: int, iz: int) -> np.ndarray:
    """Receivers on every node of the plane z=iz, x fastest then y."""
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.zeros((nx * ny, 3), dtype=np.int32)
    r[:, 0] = xx.ravel()
    r[:, 1] = yy.ravel()
    r[:, 2] = iz
    return r


@dataclass
class Workload:
    name: str
    shape: tuple           # (nz, ny, nx)
    h: float               # grid spacing (m), equal on all axes
    dt: float              # s
    nt: int
    src: tuple             # (ix, iy, iz)
    rec: np.ndarray        # int32 [nrec, 3] of (ix, iy, iz)
    f0: float              # Ricker peak frequency (Hz)
    t0: float              # Ricker delay (s)
    sponge_width: int = 0
    sponge_alpha: float = 0.015
    make_velocity: Callable[[], np.ndarray] = field(default=None, repr=False)

    @property
    def npts(self) -> int:
        nz, ny, nx = self.shape
        return nx * ny * nz

    def velocity(self) -> np.ndarray:
        return self.make_velocity()

    def wavelet(self, nt: int | None = None) -> np.ndarray:
        return ricker(self.nt if nt is None else nt, self.dt, self.f0, self.t0)


def _small() -> Workload:
    n = 64
    return Workload(
        name="small-64^3", shape=(n, n, n), h=10.0, dt=COURANT * 10.0 / V.V_MAX, nt=200,
        src=(32, 32, 32), rec=line_receivers(n, 32, 4), f0=15.0, t0=1.0 / 15.0,
        sponge_width=0, make_velocity=lambda: V.smooth_random((n, n, n), seed=1))


def _large() -> Workload:
    n = 512
    return Workload(
        name="large-512^3", shape=(n, n, n), h=10.0, dt=COURANT * 10.0 / V.V_MAX, nt=1000,
        src=(256, 256, 10), rec=plane_receivers(n, n, 0), f0=15.0, t0=1.0 / 15.0,
        sponge_width=20, sponge_alpha=0.015,
        make_velocity=lambda: V.layered_perturbed((n, n, n), seed=2))


def _precision() -> Workload:
    n = 1024
    return Workload(
        name="precision-1024^3", shape=(n, n, n), h=10.0, dt=COURANT * 10.0 / V.V_MAX, nt=500,
        src=(512, 512, 512), rec=line_receivers(n, 512, 4), f0=15.0, t0=1.0 / 15.0,
        sponge_width=0, make_velocity=None)  # built on the device: smooth_random_torch(seed=3)


def _precision_crop() -> Workload:
    n, full, o = 128, 1024, 448
    return Workload(
        name="precision-crop-128^3", shape=(n, n, n), h=10.0, dt=COURANT * 10.0 / V.V_MAX, nt=500,
        src=(64, 64, 64), rec=line_receivers(n, 64, 4), f0=15.0, t0=1.0 / 15.0, sponge_width=0,
        make_velocity=lambda: V.smooth_random((n, n, n), seed=3, origin=(o, o, o),
                                              full_shape=(full, full, full)))


def _gradient(n: int = 256) -> Workload:
    iface = 48 * n // 256
    return Workload(
        name=f"gradient-{n}^3", shape=(n, n, n), h=10.0, dt=COURANT * 10.0 / 3000.0, nt=800,
        src=(n // 2, n // 2, 4), rec=plane_receivers(n, n, 4), f0=10.0, t0=0.1, sponge_width=0,
        make_velocity=lambda: V.two_layer((n, n, n), iface))


WORKLOADS = {
    "small": _small,
    "large": _large,
    "precision": _precision,
    "precision_crop": _precision_crop,
    "gradient": _gradient,
}


def workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)


def serving_requests(count: int = 512, rate: float = 20.0, seed: int = 5):
    """Poisson arrivals of independent forward shots (one dict per request)."""
    rng = np.random.default_rng(seed)
    grids = [(128, 128, 128), (128, 192, 256), (256, 256, 256), (384, 384, 384)]  # (nz, ny, nx)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        nz, ny, nx = grids[int(rng.integers(0, len(grids)))]
        nt = int(rng.integers(500, 2001))
        storage = "f16" if rng.uniform() < 0.5 else "f32"
        out.append(dict(id=i, arrival=float(arrivals[i]), shape=(nz, ny, nx), nt=nt, storage=storage,
                        h=10.0, dt=COURANT * 10.0 / V.V_MAX, src=(nx // 2, ny // 2, 4),
                        rec=line_receivers(nx, ny // 2, 4), f0=15.0, t0=1.0 / 15.0,
                        sponge_width=20, sponge_alpha=0.015, velocity_seed=5000 + i))
    return out
