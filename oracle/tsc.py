"""TEST INFRASTRUCTURE -- CPU reference of the triangle-shaped-cloud (TSC) density
assignment and force interpolation (Sec. VI.C), in numpy float64.

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py`` may use it; it shares
nothing with the GPU library.

Conventions (box units, periodic): the box is [0, 1) per axis on an N^3 grid, cell i covering
[i/N, (i+1)/N) with its centre at (i + 1/2)/N.  A particle at x has s = x N (taken modulo N);
its nearest cell centre is that of cell floor(s), at offset d = s - floor(s) - 1/2 in [-1/2,
1/2) cells.  The TSC cloud (a triangle two cells wide, Hockney & Eastwood) gives the three
cells floor(s) - 1, floor(s), floor(s) + 1 the weights
    W(-1) = (1/2 - d)^2 / 2,   W(0) = 3/4 - d^2,   W(+1) = (1/2 + d)^2 / 2
per axis, and the product of the three axes in 3-D.  The density of a cell is the sum of the
particle masses times their weights (cell volume 1 in cell units, so N^3 particles of mass 1
give mean density 1).  The force on a particle is the same weights applied to the cell
accelerations g = -grad phi, the gradient taken by central differences, g_x = -(phi[i+1] -
phi[i-1]) N / 2, so that assignment and interpolation are the same operator (momentum
conservation, Sec. VI.C).
"""
from __future__ import annotations

import numpy as np


def _cells_and_weights(pos, N):
    """Nearest-centre cell index (int64, shape (np, 3)) and the per-axis weights (np, 3, 3):
    w[:, axis, t] for offsets t - 1 = -1, 0, +1."""
    s = np.mod(np.asarray(pos, dtype=np.float64) * N, N)
    i = np.floor(s)
    d = s - i - 0.5
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=-1)
    return i.astype(np.int64) % N, w


def deposit(pos, N: int, mass: float = 1.0) -> np.ndarray:
    """TSC density on the periodic N^3 grid of particles at pos (np, 3) in [0, 1)."""
    idx, w = _cells_and_weights(pos, N)
    rho = np.zeros((N, N, N))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                val = mass * w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                np.add.at(rho, ((idx[:, 0] + a - 1) % N, (idx[:, 1] + b - 1) % N, (idx[:, 2] + c - 1) % N), val)
    return rho


def cell_acceleration(phi) -> np.ndarray:
    """g = -grad phi at the cells by central differences, shape (3, N, N, N)."""
    phi = np.asarray(phi, dtype=np.float64)
    N = phi.shape[0]
    return np.stack([-(np.roll(phi, -1, axis=ax) - np.roll(phi, 1, axis=ax)) * (N / 2.0) for ax in range(3)])


def interpolate(field, pos) -> np.ndarray:
    """TSC interpolation of a cell field (C, N, N, N) to the particles: (np, C)."""
    field = np.asarray(field, dtype=np.float64)
    N = field.shape[-1]
    idx, w = _cells_and_weights(pos, N)
    out = np.zeros((len(idx), field.shape[0]))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                wt = w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                cell = ((idx[:, 0] + a - 1) % N, (idx[:, 1] + b - 1) % N, (idx[:, 2] + c - 1) % N)
                out += wt[:, None] * field[:, cell[0], cell[1], cell[2]].T
    return out


def force(phi, pos) -> np.ndarray:
    """Acceleration -grad phi interpolated to the particles with the TSC weights: (np, 3)."""
    return interpolate(cell_acceleration(phi), pos)
