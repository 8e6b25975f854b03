"""Pins of the oracle's truncation-error estimate tau^h = L^H(R u) - R L^h(u) (Sec. V.B),
CPU only.  tau measures how far the coarse operator is from the restricted fine one:
- it vanishes for a uniform state (every term of both operators is then the same constant);
- for a smooth field it is the difference of two second-order discretisations, so it falls
  as h^2 when the grid is refined at fixed physical field;
- the density and background terms cancel: tau does not change when a uniform offset is
  added to rho~ (rho_ref moved along), since both levels subtract the same source.
"""
import numpy as np
import pytest

import oracle as O
import paper_refs as R


def _model():
    return O.Model(box_mpc_h=64.0, fr0_abs=1e-5)


def smooth_u(model, N, amp=0.5):
    x = (np.arange(N) + 0.5) / N
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return R.ubar(model) + amp * (np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.5 * np.sin(4 * np.pi * Z))


def test_tau_vanishes_for_uniform_state():
    m = _model()
    N = 16
    u = np.full((N, N, N), R.ubar(m) + 0.3)
    rho = np.full((N, N, N), 2.5)
    t = O.tau(u, rho, m)
    L, _ = O.operator(u, m, 1.0 / N, rho=rho)
    assert np.abs(t).max() <= 1e-12 * max(1.0, np.abs(L).max())


def test_tau_falls_as_h_squared():
    m = _model()
    rms = []
    for N in (32, 64, 128):
        u = smooth_u(m, N, amp=0.1)
        rho = np.ones((N, N, N))
        rms.append(np.sqrt(np.mean(O.tau(u, rho, m) ** 2)))
    r1, r2 = rms[0] / rms[1], rms[1] / rms[2]
    assert 3.7 < r1 < 4.3 and 3.85 < r2 < 4.15, rms


def test_tau_independent_of_density_offset():
    m = _model()
    N = 16
    u = smooth_u(m, N, amp=0.2)
    rho = 1.0 + np.random.default_rng(3).uniform(0.0, 2.0, (N, N, N))
    t1 = O.tau(u, rho, m, rho_ref=1.0)
    t2 = O.tau(u, rho + 5.0, m, rho_ref=6.0)
    scale = np.abs(t1).max()
    np.testing.assert_allclose(t1, t2, rtol=0, atol=1e-9 * scale)


def test_tau_of_a_small_mode_matches_its_linearisation():
    """u = u_bar + eps cos(2 pi x), rho~ = 1.  To first order in eps only the flux term
    contributes: it is c~^2 b_bar times the 7-point Laplacian (b = e^u_bar), the 8-child mean
    of the mode is cos(pi h) times the mode at the coarse centre, and the Laplacians act on
    it with their eigenvalues lambda_h = (2 cos(2 pi h) - 2)/h^2 and lambda_H likewise with
    H = 2h.  So tau = eps c~^2 b_bar cos(pi h) (lambda_H - lambda_h) cos(2 pi x_c): positive
    where the mode is, since the coarse operator's truncation error is four times the fine
    one's."""
    m = _model()
    N, eps = 32, 1e-5
    h, H = 1.0 / N, 2.0 / N
    x = (np.arange(N) + 0.5) * h
    u = R.ubar(m) + eps * np.cos(2 * np.pi * x)[:, None, None] * np.ones((1, N, N))
    t = O.tau(u, np.ones((N, N, N)), m)
    xc = (np.arange(N // 2) + 0.5) * H
    lam_h = (2 * np.cos(2 * np.pi * h) - 2) / h ** 2
    lam_H = (2 * np.cos(2 * np.pi * H) - 2) / H ** 2
    expect = eps * R.ctilde(m) ** 2 * np.exp(R.ubar(m)) * np.cos(np.pi * h) * (lam_H - lam_h) * np.cos(2 * np.pi * xc)
    np.testing.assert_allclose(t, expect[:, None, None] * np.ones((1, N // 2, N // 2)), rtol=2e-3,
                               atol=2e-3 * np.abs(expect).max())
