"""Pins of the oracle's refinement level with the mask scheme (Sec. V: masks, eq. phi_b,
eq. u_i-1jk, eq. bc_modified_fR_op, eq. bc_modified_fR_dop, and the masked restriction and
prolongation rules of Sec. V.A.2, V.A.3 and V.B.2), checked against things other than the
oracle's own masked code:

* the operator against the paper's expanded form of the BC-modified equation and of its
  derivative, written out term by term (a different algebraic route from the oracle's ghost
  substitution), on fractional masks with several masked faces per cell;
* the derivative against central finite differences of the operator;
* an all-active mask against the oracle's periodic domain solve;
* a cube-shaped active region against the oracle's cube-patch solve, whose boundary values
  are u_b = (w_ghost + w_face) / 2 (eq. phi_b with masks -1 and +1);
* the converged field on an irregular oct mask against plain single-grid relaxation of the
  same fine-level equations (the coarse-level rules change only the path, not the fixed
  point), and the V-cycle's convergence factor on that mask.
"""
import numpy as np
import pytest

import oracle as O
from paper_1110_1379_amd import inputs

MODEL = O.Model(box_mpc_h=32.0, fr0_abs=1e-5)


def expanded_operator(u, w, mask, model, rho=None, rho_ref=1.0):
    """eq. bc_modified_fR_op and eq. bc_modified_fR_dop as printed, with each masked
    neighbour contributing its own (1 - r) terms (r = m_nb / m_i), one cell at a time."""
    c = O.constants(model, u.shape[0])
    C, A, D, Sbar = c["C"], c["A"], c["D"], c["Sbar"]
    npow = model.n
    n = u.shape[0]
    L = np.zeros_like(u)
    dL = np.zeros_like(u)
    mag = np.zeros_like(u)   # sum of the magnitudes of the terms: the scale of rounding
    offs = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for i, j, k in np.ndindex(n, n, n):
        mi = mask[i, j, k]
        if not mi > 0:
            continue
        ui = u[i, j, k]
        bi = np.exp(ui)
        s_u = s_b = s_bu = 0.0      # the active neighbours: sum u, sum b, sum b u
        g_u = g_b = g_bu = 0.0      # masked neighbours: (1-r) u_b, (1-r) e^..., (1-r) u_b e^...
        s_r = 0.0                   # sum of r over masked neighbours
        g_d = 0.0                   # (1-r) r e^... (u_i - u_b)
        for di, dj, dk in offs:
            p = ((i + di) % n, (j + dj) % n, (k + dk) % n)
            if mask[p] > 0:
                s_u += u[p]
                s_b += np.exp(u[p])
                s_bu += np.exp(u[p]) * u[p]
            else:
                r = mask[p] / mi
                ub = mi / (mi - mask[p]) * w[p] - mask[p] / (mi - mask[p]) * w[i, j, k]
                e = np.exp((1 - r) * ub) * np.exp(r * ui)
                g_u += (1 - r) * ub
                g_b += (1 - r) * e
                g_bu += (1 - r) * ub * e
                g_d += (1 - r) * r * e * (ui - ub)
                s_r += r
        K = (npow * model.a ** 2 * c["xi"]) ** (1 / (npow + 1))
        curv = model.omega_m * model.a ** 4 * K * np.exp(-ui / (npow + 1)) / 3.0
        assert np.isclose(curv, A * np.exp(-ui / (npow + 1)))
        val = (C * bi * (s_u + g_u - (6 - s_r) * ui) - C * ui * (s_b + g_b) + C * (s_bu + g_bu) + curv)
        if rho is not None:
            val += -D * (rho[i, j, k] - rho_ref) - Sbar
        L[i, j, k] = val
        mag[i, j, k] = (C * (bi * (abs(s_u) + abs(g_u) + 6 * abs(ui)) + abs(ui) * (s_b + g_b) + abs(s_bu) + abs(g_bu)
                             + abs(g_d)) + curv + (0.0 if rho is None else abs(D * (rho[i, j, k] - rho_ref)) + Sbar))
        dL[i, j, k] = (C * bi * (s_u + g_u - (6 - s_r) * ui) - C * (s_b + g_b) - C * (6 - s_r) * bi - C * g_d
                       - curv / (npow + 1))
    return L, dL, mag


def random_level(n, seed, fractional=True):
    rng = np.random.default_rng(seed)
    ub = O.constants(MODEL, n)["ubar"]
    u = ub + 0.3 * rng.standard_normal((n, n, n))
    w = ub + 0.3 * rng.standard_normal((n, n, n))
    if fractional:
        # restricted-mask values: multiples of 1/4 in [-1, 1], zero included
        mask = rng.integers(-4, 5, size=(n, n, n)) / 4.0
    else:
        mask = np.where(rng.random((n, n, n)) < 0.6, 1.0, -1.0)
    rho = inputs.lognormal(n, 1.0, -2.0, seed)
    return u, w, mask, rho


@pytest.mark.parametrize("fractional", [False, True])
def test_masked_operator_matches_the_expanded_equation(fractional):
    u, w, mask, rho = random_level(8, 1 + fractional, fractional)
    L, dL = O.masked_operator(u, w, mask, MODEL, rho=rho)
    Le, dLe, mag = expanded_operator(u, w, mask, MODEL, rho=rho)
    act = mask > 0
    assert act.sum() > 50
    # a few hundred units in the last place of the summed term magnitudes (the expanded
    # form cancels terms of size |u| C sum b)
    assert np.all(np.abs(L - Le) <= 1e-13 * mag)
    assert np.all(np.abs(dL - dLe) <= 1e-13 * mag)
    assert np.all(L[~act] == 0) and np.all(dL[~act] == 0)
    # coarse-level form (no density or background terms)
    L0, _ = O.masked_operator(u, w, mask, MODEL)
    L0e, _, mag0 = expanded_operator(u, w, mask, MODEL)
    assert np.all(np.abs(L0 - L0e) <= 1e-13 * mag0)


def test_masked_derivative_is_the_finite_difference():
    u, w, mask, rho = random_level(8, 5, True)
    _, dL = O.masked_operator(u, w, mask, MODEL, rho=rho)
    ii, jj, kk = np.indices(u.shape)
    eps = 1e-6
    for colour in (0, 1):
        sel = ((ii + jj + kk) % 2 == colour)
        # cells of one colour have neighbours of the other only: L_i sees only its own shift
        Lp, _ = O.masked_operator(u + eps * sel, w, mask, MODEL, rho=rho)
        Lm, _ = O.masked_operator(u - eps * sel, w, mask, MODEL, rho=rho)
        fd = (Lp - Lm) / (2 * eps)
        act = sel & (mask > 0)
        assert np.allclose(fd[act], dL[act], rtol=1e-6, atol=1e-6 * np.abs(dL[act]).max())


@pytest.mark.parametrize("N", [16, 32])
def test_all_active_mask_is_the_domain_solve(N):
    rho = inputs.small_box(N, 2)
    ub = O.constants(MODEL, N)["ubar"]
    u1, h1, s1 = O.solve_masked(rho, np.ones_like(rho), MODEL, np.full_like(rho, ub), O.Opts(tol=1e-12))
    u2, h2, s2 = O.solve(rho, MODEL, O.Opts(tol=1e-12))
    assert s1 == 0 and s2 == 0
    assert len(h1) == len(h2)
    assert np.allclose(h1, h2, rtol=1e-8, atol=1e-13)
    assert np.abs(u1 - u2).max() <= 1e-12


def test_cube_region_is_the_cube_patch_solve():
    N, n, o = 32, 16, 8
    rho = inputs.small_box(N, 3)
    ub = O.constants(MODEL, N)["ubar"]
    w = ub + 0.5 * inputs.gaussian_field(N, 1.0, -2.0, seed=9)
    mask = -np.ones((N, N, N))
    sl = (slice(o, o + n),) * 3
    mask[sl] = 1.0
    um, hm, sm = O.solve_masked(rho, mask, MODEL, w, O.Opts(tol=1e-11))
    assert sm == 0
    assert np.array_equal(um[mask < 0], w[mask < 0])
    # cube patch: faces -x,+x,-y,+y,-z,+z with u_b = (w_ghost + w_face) / 2
    wi = w[sl]
    faces = np.zeros((6, n, n))
    faces[0] = 0.5 * (w[o - 1, o:o + n, o:o + n] + wi[0])
    faces[1] = 0.5 * (w[o + n, o:o + n, o:o + n] + wi[-1])
    faces[2] = 0.5 * (w[o:o + n, o - 1, o:o + n] + wi[:, 0])
    faces[3] = 0.5 * (w[o:o + n, o + n, o:o + n] + wi[:, -1])
    faces[4] = 0.5 * (w[o:o + n, o:o + n, o - 1] + wi[:, :, 0])
    faces[5] = 0.5 * (w[o:o + n, o:o + n, o + n] + wi[:, :, -1])
    up, hp, sp = O.solve_patch(rho[sl], 1.0 / N, faces, MODEL, wi, O.Opts(tol=1e-11))
    assert sp == 0
    assert np.abs(um[sl] - up).max() <= 1e-11


def irregular_level(N, seed):
    rho = inputs.small_box(N, seed)
    od = rho.reshape(N // 2, 2, N // 2, 2, N // 2, 2).mean(axis=(1, 3, 5))
    mask = inputs.oct_mask(rho, float(np.quantile(od, 0.9)), expand=1)
    ub = O.constants(MODEL, N)["ubar"]
    u0 = ub + 0.5 * inputs.gaussian_field(N, 1.0, -2.0, seed=seed + 20)
    return rho, mask, u0


def test_irregular_mask_fixed_point_is_the_single_grid_one():
    N = 16
    rho, mask, u0 = irregular_level(N, 1)
    assert 0.2 < (mask > 0).mean() < 0.8
    u_mg, h_mg, st = O.solve_masked(rho, mask, MODEL, u0, O.Opts(tol=1e-11, coarsest_n=2))
    assert st == 0
    # one level only: the coarsest-level relaxation is plain red-black Newton-Gauss-Seidel
    sg = O.Opts(tol=1e-11, coarsest_n=N, coarsest_sweeps=20000, coarsest_rtol=1e-14, max_cycles=3)
    u_sg, h_sg, st_sg = O.solve_masked(rho, mask, MODEL, u0, sg)
    assert st_sg == 0, h_sg
    assert np.abs(u_mg - u_sg).max() <= 1e-10
    # other sweep counts, other path, same field
    u_b, _, st_b = O.solve_masked(rho, mask, MODEL, u0, O.Opts(tol=1e-11, pre=1, post=3, coarsest_n=4))
    assert st_b == 0 and np.abs(u_b - u_mg).max() <= 1e-10


def test_irregular_mask_converges_at_a_multigrid_rate_and_keeps_masked_cells():
    N = 32
    rho, mask, u0 = irregular_level(N, 0)
    u, h, st = O.solve_masked(rho, mask, MODEL, u0, O.Opts(tol=1e-12))
    assert st == 0
    assert np.array_equal(u[mask < 0], u0[mask < 0])
    rates = h[2:-1] / h[1:-2]
    assert rates.max() <= 0.25, rates
    # the rms is over active cells only: recompute it from the operator
    L, _ = O.masked_operator(u, u0, mask, MODEL, rho=rho)
    assert np.isclose(np.sqrt(np.mean(L[mask > 0] ** 2)), h[-1], rtol=1e-6)
