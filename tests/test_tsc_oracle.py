"""Pins of the oracle's TSC density assignment and force interpolation (Sec. VI.C), against
facts that do not come from its own code:

* the weights of one particle written out by hand for a chosen offset, and their sum 1;
* a particle at every cell centre gives a density of exactly 1 everywhere;
* mass conservation: the mean density is the total mass over N^3 (the check the paper runs
  at every step: mean density 1 on the domain grid);
* a shift of every particle by whole cells shifts the density by the same cells;
* momentum conservation (the reason the paper interpolates forces with the same TSC
  weights): with phi the periodic solution of lap phi = rho - 1 for the TSC density itself,
  the forces on all particles add up to zero;
* the force of a sine potential on a particle, summed by hand from the three weights per
  axis and the central-difference gradient.
"""
import numpy as np
import pytest

from oracle import tsc
from oracle import poisson as P
from paper_1110_1379_amd import inputs


def test_single_particle_weights_by_hand():
    N = 8
    # particle 1/4 cell right of the centre of cell (3, 5, 0): offset d = 0.25 along x,
    # 0 along y, -0.5 (the cell's left edge) along z
    pos = np.array([[(3 + 0.75) / N, (5 + 0.5) / N, 0.0]])
    rho = tsc.deposit(pos, N)
    wx = {2: 0.03125, 3: 0.6875, 4: 0.28125}
    wy = {4: 0.125, 5: 0.75, 6: 0.125}
    # d = -1/2: (1/2 + 1/2)^2 / 2 = 1/2 to the left (periodic: cell 7), 3/4 - 1/4 = 1/2 to the
    # cell itself, 0 to the right
    wz = {7: 0.5, 0: 0.5, 1: 0.0}
    expect = np.zeros((N, N, N))
    for i, a in wx.items():
        for j, b in wy.items():
            for k, c in wz.items():
                expect[i, j, k] += a * b * c
    assert np.array_equal(rho, expect)
    assert rho.sum() == 1.0


def test_weights_sum_to_one():
    rng = np.random.default_rng(0)
    pos = rng.random((1000, 3))
    _, w = tsc._cells_and_weights(pos, 16)
    assert np.allclose(w.sum(axis=2), 1.0, rtol=0, atol=1e-15)
    assert np.all(w >= 0)


def test_particles_at_cell_centres_give_uniform_density():
    N = 16
    q = (np.arange(N) + 0.5) / N
    pos = np.stack(np.meshgrid(q, q, q, indexing="ij"), axis=-1).reshape(-1, 3)
    rho = tsc.deposit(pos, N)
    assert np.allclose(rho, 1.0, rtol=0, atol=1e-14)


def test_mass_conservation_and_shift():
    N = 32
    pos = inputs.particles(16, seed=1)
    m = N ** 3 / len(pos)
    rho = tsc.deposit(pos, N, m)
    assert abs(rho.mean() - 1.0) <= 1e-13
    assert rho.min() >= 0.0
    shifted = tsc.deposit(np.mod(pos + np.array([3, -2, 5]) / N, 1.0), N, m)
    assert np.allclose(shifted, np.roll(rho, (3, -2, 5), axis=(0, 1, 2)), rtol=0, atol=1e-12 * rho.max())


def test_momentum_conservation():
    N = 32
    pos = inputs.particles(16, seed=2)
    m = N ** 3 / len(pos)
    rho = tsc.deposit(pos, N, m)
    phi = P.solve(rho - 1.0)     # periodic 7-point solve, zero-mean source
    F = tsc.force(phi, pos) * m
    scale = np.abs(F).sum(axis=0)
    assert np.all(np.abs(F.sum(axis=0)) <= 1e-11 * scale)
    # a mismatched interpolation (cloud-in-cell, two cells per axis) breaks it
    idx = np.floor(np.mod(pos * N - 0.5, N)).astype(np.int64)
    d = np.mod(pos * N - 0.5, N) - idx
    g = tsc.cell_acceleration(phi)
    Fc = np.zeros_like(F)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                wt = (d[:, 0] if a else 1 - d[:, 0]) * (d[:, 1] if b else 1 - d[:, 1]) * (d[:, 2] if c else 1 - d[:, 2])
                cell = ((idx[:, 0] + a) % N, (idx[:, 1] + b) % N, (idx[:, 2] + c) % N)
                Fc += wt[:, None] * g[:, cell[0], cell[1], cell[2]].T
    assert np.any(np.abs((Fc * m).sum(axis=0)) > 1e-6 * scale)


def test_force_of_a_sine_potential_by_hand():
    N = 16
    x = np.arange(N)
    phi = np.broadcast_to(np.sin(2 * np.pi * (x + 0.5) / N)[:, None, None], (N, N, N)).copy()
    p = np.array([[(6 + 0.5 + 0.3) / N, 0.41, 0.77]])
    F = tsc.force(phi, p)
    d = 0.3
    w = [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
    gx = lambda i: -(np.sin(2 * np.pi * (i + 1.5) / N) - np.sin(2 * np.pi * (i - 0.5) / N)) * N / 2
    expect = w[0] * gx(5) + w[1] * gx(6) + w[2] * gx(7)
    assert abs(F[0, 0] - expect) <= 1e-13 * N
    assert abs(F[0, 1]) <= 1e-13 and abs(F[0, 2]) <= 1e-13
