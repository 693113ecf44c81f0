"""Velocity gradients through torch.autograd.

``wave_forward(vel, wavelet, geometry)`` returns the receiver traces of one
shot; its backward calls libwave's checkpointed adjoint (``wave_adjoint``),
so ``loss(traces).backward()`` deposits dloss/dv in ``vel.grad``.  The
forward run and the adjoint both execute in the library's HIP kernels; torch
only holds the tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from .solver import Solver


@dataclass
class Geometry:
    h: object                   # grid spacing, scalar or (dx, dy, dz)
    dt: float
    nt: int
    src: tuple                  # (ix, iy, iz)
    rec: np.ndarray             # int [nrec, 3] of (ix, iy, iz)
    sponge_width: int = 0
    sponge_alpha: float = 0.015
    ckpt_interval: int = 0      # 0: ceil(sqrt(nt))
    variant: int = 0
    options: dict = field(default_factory=dict)


class WaveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel, wavelet, geom: Geometry):
        s = Solver(vel.detach().contiguous(), geom.h, geom.dt, src=geom.src, rec=geom.rec,
                   sponge_width=geom.sponge_width, sponge_alpha=geom.sponge_alpha, adjoint=True,
                   nt_max=geom.nt, ckpt_interval=geom.ckpt_interval, variant=geom.variant, **geom.options)
        wav = wavelet.detach().contiguous()
        traces = s.run(geom.nt, wav)
        ctx.solver = s
        ctx.wavelet = wav
        ctx.nt = geom.nt
        return traces

    @staticmethod
    def backward(ctx, grad_traces):
        s = ctx.solver
        grad = s.adjoint(ctx.nt, ctx.wavelet, grad_traces.contiguous().float())
        s.close()
        ctx.solver = None
        return grad, None, None


def wave_forward(vel: torch.Tensor, wavelet: torch.Tensor, geom: Geometry) -> torch.Tensor:
    return WaveFn.apply(vel, wavelet, geom)
