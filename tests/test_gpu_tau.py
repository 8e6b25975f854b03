"""Parity of the GPU truncation-error estimate (mgfr_tau) with the oracle's tau (Sec. V.B,
the FAS relation tau^h = L^H(R u) - R L^h(u)), and the tau-based stop rule of the domain
solve (opts.tau_alpha), on an MI355X.

Fields are seeded and synthetic (never taken from the GPU path): a rough u = u_bar + 0.3 n
(n unit normal per cell) on a lognormal density, and at 512^3 the halo density of the
benchmark with a smooth Gaussian u.  tau is a difference of operator values of size up to
12 C max e^u, so the bar is 1e-13 of that scale per element, as for the residual.  Sizes 16
and 32 run the unfused restriction, 64 and above the streaming residual-restriction pass.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1110_1379_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    from paper_1110_1379_amd import mgfr
    assert torch.cuda.is_available()
    mgfr.lib()
    return mgfr


@pytest.fixture(scope="module")
def ctx(mg):
    c = mg.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def op_scale(m, N, u, rho):
    C = O.constants(m, N)["C"]
    return 12 * C * np.exp(u).max() * 2.0 + 0.24 * np.abs(rho).max() + 4.0


@pytest.mark.parametrize("N,subtract_mean", [(16, False), (32, True), (64, False), (128, True), (256, False)])
def test_tau_matches_oracle(mg, ctx, N, subtract_mean):
    say(f"[tau] N={N} subtract_mean={subtract_mean}")
    box = 64.0 if N <= 64 else float(N)
    p = mg.Params(box_mpc_h=box, fr0_abs=1e-5)
    m = O.Model(box_mpc_h=box, fr0_abs=1e-5)
    rho = inputs.lognormal(N, 1.5, -2.0, seed=N + 1)
    u = O.constants(m, N)["ubar"] + 0.3 * np.random.default_rng(N).standard_normal((N, N, N))
    flags = mg.MGFR_SUBTRACT_MEAN if subtract_mean else 0
    tau, rms = mg.mgfr_tau(ctx, dev(rho), dev(u), p, flags=flags)
    ref = O.tau(u, rho, m, rho_ref=rho.mean() if subtract_mean else 1.0)
    g = tau.cpu().numpy()
    assert g.shape == (N // 2,) * 3
    err = np.abs(g - ref).max()
    scale = op_scale(m, N, u, rho)
    rms_ref = np.sqrt(np.mean(ref ** 2))
    say(f"  max err {err:.2e} (bar {1e-13 * scale:.2e}), rms {rms:.6e} vs {rms_ref:.6e}")
    assert err <= 1e-13 * scale
    assert abs(rms - rms_ref) <= 1e-10 * rms_ref


def test_tau_full_size_sampled(mg, ctx):
    """512^3 halo density (the benchmark's box, 512 Mpc/h, |f_R0| = 1e-6) with a smooth
    Gaussian u: tau at 4096 sampled coarse cells from the oracle's pointwise operator on the
    restricted and on the fine field."""
    say("[tau] full size 512 sampled")
    N, box, fr0 = 512, 512.0, 1e-6
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    rho = inputs.halo_box(N)
    u = O.constants(m, N)["ubar"] + inputs.gaussian_field(N, 1.0, -2.0, seed=5)
    tau, rms = mg.mgfr_tau(ctx, dev(rho), dev(u), p)
    g = tau.cpu().numpy()
    del tau
    Ru, Rrho = O.restrict_mean(u), O.restrict_mean(rho)
    rng = np.random.default_rng(3)
    n = N // 2
    Q = rng.integers(0, n, size=(4096, 3))
    LH = O.operator_at(Ru, m, 2.0 / N, (Q[:, 0] * n + Q[:, 1]) * n + Q[:, 2], rho=Rrho)
    del Ru, Rrho
    Lh = np.zeros(len(Q))
    for a in range(2):
        for b in range(2):
            for z in range(2):
                F = 2 * Q + np.array([a, b, z])
                Lh += O.operator_at(u, m, 1.0 / N, (F[:, 0] * N + F[:, 1]) * N + F[:, 2], rho=rho)
    ref = LH - Lh / 8.0
    got = g[Q[:, 0], Q[:, 1], Q[:, 2]]
    err = np.abs(got - ref).max()
    scale = op_scale(m, N, u, rho)
    say(f"  sampled max err {err:.2e} (bar {1e-13 * scale:.2e}), rms {rms:.4e}")
    assert err <= 1e-13 * scale
    assert np.isclose(rms, np.sqrt(np.mean(g ** 2)), rtol=1e-10)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tau_stop_rule(mg, ctx, precision):
    """With a tolerance below what double precision reaches, the solve still ends: it stops
    at the first cycle whose rms residual is <= tau_alpha x rms(tau), and the reported rms(tau)
    is that of the oracle's tau on the returned field."""
    say(f"[tau] stop rule {precision}")
    N, alpha = 64, 1.0 / 3.0
    p = mg.Params(box_mpc_h=64.0, fr0_abs=1e-5)
    m = O.Model(box_mpc_h=64.0, fr0_abs=1e-5)
    rho = inputs.small_box(N, 0)
    prec = mg.MGFR_FP64 if precision == "fp64" else mg.MGFR_MIXED
    o = mg.mgfr_default_opts(tol=1e-30, max_cycles=40, precision=prec, tau_alpha=alpha)
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, o)
    assert st == mg.MGFR_OK, ctx.last_error()
    stats = mg.mgfr_get_stats(ctx)
    t = stats["tau_rms"]
    u = u_d.cpu().numpy()
    ref_t = np.sqrt(np.mean(O.tau(u, rho, m) ** 2))
    L, _ = O.operator(u, m, 1.0 / N, rho=rho)
    ref_r = np.sqrt(np.mean(L ** 2))
    say(f"  cycles {len(hist) - 1}, rms {hist[-1]:.3e} (oracle {ref_r:.3e}), tau rms {t:.3e} (oracle {ref_t:.3e})")
    assert abs(t - ref_t) <= 1e-8 * ref_t
    assert hist[-1] <= alpha * t
    assert abs(ref_r - hist[-1]) <= 1e-3 * hist[-1]
    # the cycle before did not pass (tau changes little between the last cycles)
    assert len(hist) >= 2 and hist[-2] > 0.5 * alpha * t
    # without the rule the same tolerance is never met
    o2 = mg.mgfr_default_opts(tol=1e-30, max_cycles=len(hist) + 1, precision=prec)
    _, _, st2 = mg.mg_fr_solve(ctx, dev(rho), p, o2)
    assert st2 == mg.MGFR_ENOTCONV
    assert mg.mgfr_get_stats(ctx)["tau_rms"] == 0.0


def test_tau_errors(mg, ctx):
    say("[tau] errors")
    p = mg.Params(box_mpc_h=64.0, fr0_abs=1e-5)
    x = dev(np.ones((6, 6, 6)))
    with pytest.raises(mg.MgfrError):
        mg.mgfr_tau(ctx, x, x, p)
