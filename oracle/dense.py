"""Brute-force dense matrix of the Laplacian of Eq. 1 (FP64, tiny grids).

Built by explicit loops over every node and every stencil tap with bounds
checks (a neighbour outside the grid contributes nothing), independent of
the slicing in ``operators.laplacian``.
"""
from __future__ import annotations

import numpy as np

from .coefficients import second_derivative_weights


def dense_laplacian(shape, h) -> np.ndarray:
    """N x N matrix, N = nx ny nz, rows/cols in flat order x + nx (y + ny z)."""
    nz, ny, nx = shape
    hx, hy, hz = (h, h, h) if np.isscalar(h) else h
    c = second_derivative_weights(4)
    N = nx * ny * nz
    A = np.zeros((N, N), dtype=np.float64)

    def flat(x, y, z):
        return x + nx * (y + ny * z)

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                row = flat(x, y, z)
                for axis, ha in ((0, hx), (1, hy), (2, hz)):
                    w = 1.0 / (ha * ha)
                    A[row, row] += c[0] * w
                    for m in range(1, 5):
                        for sgn in (1, -1):
                            q = [x, y, z]
                            q[axis] += sgn * m
                            if 0 <= q[0] < nx and 0 <= q[1] < ny and 0 <= q[2] < nz:
                                A[row, flat(*q)] += c[m] * w
    return A
