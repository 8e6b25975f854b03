"""Pins of the modified Poisson oracle (oracle/poisson.py) against what the paper and the
mathematics fix, independently of the oracle's own formulas (CPU only).

- solve: the returned phi satisfies the 7-point stencil applied directly in the test
  (a different computation from the Fourier-space solve), has zero mean, and for a smooth
  mode converges at O(h^2) to the continuum solution -f/(4 pi^2 |k|^2).
- source: the three regimes of Sec. II. At the background (rho~ = 1, u = u_bar) the source
  vanishes. Where the scalaron stays at its background value, delta R = 0 and the source is
  4/3 of the GR one. For a uniform overdensity in the GR-restored state, delta R = 8 pi G
  delta rho and the source equals the GR one, (3/2) Om a (rho~ - 1) in code units. u_bar
  and the GR-restored u come from the paper's background relations in paper_refs, not from
  the oracle.
"""
import numpy as np
import pytest

import oracle as O
from oracle import poisson as P

import paper_refs as R


def stencil(phi):
    """Written out here as the plain 7-point sum, on index arithmetic."""
    N = phi.shape[0]
    out = np.empty_like(phi)
    idx = np.arange(N)
    up, dn = (idx + 1) % N, (idx - 1) % N
    out[:] = (phi[up, :, :] + phi[dn, :, :] + phi[:, up, :] + phi[:, dn, :] + phi[:, :, up] + phi[:, :, dn]
              - 6.0 * phi)
    return out * N * N


@pytest.mark.parametrize("N", [8, 16, 32])
def test_solution_satisfies_stencil(N):
    rng = np.random.default_rng(N)
    S = rng.standard_normal((N, N, N)) * 3.0 + 0.7
    phi = P.solve(S)
    r = stencil(phi) - (S - S.mean())
    assert np.abs(r).max() <= 1e-11 * np.abs(S).max()
    assert abs(phi.mean()) <= 1e-14 * np.abs(phi).max() + 1e-300


def test_smooth_mode_converges_to_continuum():
    """f = sin(2 pi (x + 2 y)) at cell centres: the continuum solution of lap phi = f is
    -f / (4 pi^2 * 5); the discrete one approaches it at O(h^2)."""
    errs = []
    for N in (16, 32, 64):
        x = (np.arange(N) + 0.5) / N
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        f = np.sin(2 * np.pi * (X + 2 * Y))
        phi = P.solve(f)
        errs.append(np.abs(phi - (-f / (4 * np.pi ** 2 * 5))).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 < r1 < 4.3 and 3.9 < r2 < 4.1, errs


def _model(fr0=1e-5, a=1.0):
    return O.Model(box_mpc_h=64.0, fr0_abs=fr0, a=a)


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_source_vanishes_at_background(a):
    m = _model(a=a)
    N = 8
    u = np.full((N, N, N), R.ubar(m))
    S = P.source(np.ones((N, N, N)), u, m)
    scale = 2 * m.omega_m * a
    assert np.abs(S).max() <= 1e-12 * scale


def test_source_unscreened_is_four_thirds_of_gr():
    m = _model()
    N = 8
    rho = 1.0 + np.random.default_rng(1).uniform(-0.5, 3.0, (N, N, N))
    u = np.full((N, N, N), R.ubar(m))
    S = P.source(rho, u, m)
    gr = 1.5 * m.omega_m * m.a * (rho - 1.0)
    np.testing.assert_allclose(S, (4.0 / 3.0) * gr, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("c", [3.0, 50.0, 400.0])
@pytest.mark.parametrize("a", [1.0, 0.7])
def test_source_gr_restored_is_gr(c, a):
    m = _model(a=a)
    N = 4
    u = np.full((N, N, N), R.u_uniform(m, c))
    S = P.source(np.full((N, N, N), c), u, m)
    np.testing.assert_allclose(S, 1.5 * m.omega_m * a * (c - 1.0), rtol=1e-11)
