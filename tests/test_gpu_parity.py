"""Parity of the HIP library against the FP64 CPU oracle (needs an MI355X).

Bar (stated with each test): the relative field error max|u - u*| / max|u*| of the FP64
solver is <= 1e-10 with both sides converged to rms(L) <= 1e-12 (or the FP64 floor of the
case); operator values agree to rounding.  Cases span one to many workgroups and ragged
ones (N = 4 ... 64); full-size cases are checked through the oracle's operator on the GPU
solution (a property that holds at any size).
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgfr.lib()          # fails loudly if the HIP library is missing
    return mgfr


@pytest.fixture(scope="module")
def ctx(mg):
    c = mg.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def both(box, fr0, **kw):
    from paper_1110_1379_amd import mgfr
    return mgfr.Params(box_mpc_h=box, fr0_abs=fr0, **kw), O.Model(box_mpc_h=box, fr0_abs=fr0, **kw)


def rel_err(u, ref):
    return np.abs(u - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("N,box,fr0", [(16, 32.0, 1e-5), (32, 512.0, 1e-6), (64, 64.0, 1e-4)])
def test_constants_match_oracle(mg, N, box, fr0):
    p, m = both(box, fr0)
    a = mg.mgfr_constants(p, N)
    b = O.constants(m, N)
    for k in b:
        assert a[k] == pytest.approx(b[k], rel=1e-14), k


@pytest.mark.parametrize("N", [4, 8, 16, 32, 64])
def test_operator_matches_oracle(mg, ctx, N):
    say(f"[operator] N={N}")
    p, m = both(64.0, 1e-5)
    rho = inputs.lognormal(N, 1.5, -2.0, seed=N)
    ub = O.constants(m, N)["ubar"]
    u = ub + 0.3 * np.random.default_rng(N).standard_normal((N, N, N))
    d = mg.mgfr_residual(ctx, dev(rho), dev(u), p).cpu().numpy()
    L, _ = O.operator(u, m, 1.0 / N, rho=rho)
    C = O.constants(m, N)["C"]
    scale = 12 * C * np.exp(u).max() * 2.0 + 0.24 * np.abs(rho).max() + 4.0
    assert np.abs(d - L).max() <= 1e-13 * scale


@pytest.mark.parametrize("N", [64, 128])
def test_fused_sweep_is_bitwise_the_two_pass_sweep(mg, ctx, N):
    """The fused red-black sweep (redundant ring of red updates per tile) gives exactly the
    same bits as sweeping all red cells, then all black cells."""
    say(f"[smooth] fused vs two-pass N={N}")
    p, m = both(float(N), 1e-5)
    rho = inputs.lognormal(N, 2.0, -1.5, seed=11)
    u0 = O.constants(m, N)["ubar"] + 0.2 * np.random.default_rng(1).standard_normal((N, N, N))
    a = mg.mgfr_smooth(ctx, dev(rho), dev(u0), p, nsweeps=3, variant=1).cpu().numpy()
    b = mg.mgfr_smooth(ctx, dev(rho), dev(u0), p, nsweeps=3, variant=2).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("N,variant", [(16, 1), (64, 1), (64, 2)])
def test_smoother_matches_oracle_single_grid(mg, ctx, N, variant):
    """Three single-grid Newton-Gauss-Seidel sweeps against the oracle's, cell by cell."""
    say(f"[smooth] vs oracle N={N} variant={variant}")
    p, m = both(64.0, 1e-5)
    rho = inputs.lognormal(N, 1.5, -2.0, seed=12)
    u0 = O.constants(m, N)["ubar"] + 0.2 * np.random.default_rng(2).standard_normal((N, N, N))
    g = mg.mgfr_smooth(ctx, dev(rho), dev(u0), p, nsweeps=3, variant=variant).cpu().numpy()
    ref, _ = O.single_grid(rho, m, u0, 3, max_step=1.0)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()


SOLVE_CASES = [
    # (name, N, box, fr0, density maker, tol)
    ("lognormal-32-F5", 32, 64.0, 1e-5, lambda N: inputs.small_box(N, 0), 1e-12),
    ("lognormal-16-F5", 16, 32.0, 1e-5, lambda N: inputs.small_box(N, 3), 1e-12),
    # c~^2 b / h^2 ~ 220 here: the double-precision floor of the residual is ~1e-12
    ("lognormal-8-F4", 8, 16.0, 1e-4, lambda N: inputs.lognormal(N, 1.0, -2.0, 5), 1e-11),
    ("tophat-64-F5", 64, 64.0, 1e-5, lambda N: inputs.tophat_box(N, 1, count=3), 1e-11),
    ("halo-64-F6", 64, 64.0, 1e-6, lambda N: inputs.halo_box(N, 2, count=4), 1e-11),
    ("lognormal-128-F5", 128, 128.0, 1e-5, lambda N: inputs.lognormal(N, 1.5, -1.5, 6), 1e-11),
]


@pytest.mark.parametrize("name,N,box,fr0,make,tol", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_fp64_solve_matches_oracle(mg, ctx, name, N, box, fr0, make, tol):
    say(f"[solve] {name}")
    p, m = both(box, fr0)
    rho = make(N)
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, mg.mgfr_default_opts(tol=tol))
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    u_ref, h_ref, st_ref = O.solve(rho, m, O.Opts(tol=tol))
    assert st_ref == 0
    u = u_d.cpu().numpy()
    assert rel_err(u, u_ref) <= 1e-10
    # same iteration up to rounding: same number of cycles, and histories that agree to
    # six digits above the double-precision noise of the residual (~1e-13 .. 1e-12 here)
    assert len(hist) == len(h_ref)
    np.testing.assert_allclose(hist, h_ref, rtol=1e-6, atol=100 * tol)


MIXED_CASES = [
    ("lognormal-32-F5", 32, 64.0, 1e-5, lambda N: inputs.small_box(N, 0)),
    ("halo-64-F6", 64, 64.0, 1e-6, lambda N: inputs.halo_box(N, 2, count=4)),
    ("tophat-128-F5", 128, 128.0, 1e-5, lambda N: inputs.tophat_box(N, 1, count=25)),
]


@pytest.mark.parametrize("inner", [1, 2, 3])
@pytest.mark.parametrize("name,N,box,fr0,make", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_solve_matches_fp64_oracle(mg, ctx, name, N, box, fr0, make, inner):
    """Single-precision correction V-cycles inside the double-precision defect-correction loop
    reach rms(L) <= 1e-8 with max|u - u*|/max|u*| <= 1e-6 against the oracle at 1e-12."""
    say(f"[mixed] {name} inner={inner}")
    p, m = both(box, fr0)
    rho = make(N)
    o = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED, inner_cycles=inner)
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, o)
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    assert hist[-1] <= 1e-8
    u_ref, _, st_ref = O.solve(rho, m, O.Opts(tol=1e-12 if N < 128 else 1e-11))
    assert st_ref == 0
    assert rel_err(u_d.cpu().numpy(), u_ref) <= 1e-6
    # the outer residual falls at every step
    assert np.all(np.diff(hist) < 0), hist


def test_uniform_density_gives_background(mg, ctx):
    say("[solve] uniform")
    p, m = both(64.0, 1e-5)
    N = 16
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(np.ones((N, N, N))), p, mg.mgfr_default_opts(tol=1e-13))
    assert st == mg.MGFR_OK
    np.testing.assert_allclose(u_d.cpu().numpy(), O.constants(m, N)["ubar"], rtol=1e-14)


def test_subtract_mean_and_warm_start(mg, ctx):
    say("[solve] subtract-mean + warm start")
    p, m = both(64.0, 1e-5)
    N = 16
    rho = 1.7 * inputs.small_box(N, 4)               # mean 1.7: contrast about the mean
    o = mg.mgfr_default_opts(tol=1e-12, flags=mg.MGFR_SUBTRACT_MEAN)
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, o)
    assert st == mg.MGFR_OK
    u_ref, _, st_ref = O.solve(rho, m, O.Opts(tol=1e-12, subtract_mean=True))
    assert st_ref == 0
    assert rel_err(u_d.cpu().numpy(), u_ref) <= 1e-10
    # warm start from the solution: converged before the first cycle
    o2 = mg.mgfr_default_opts(tol=1e-11, flags=mg.MGFR_SUBTRACT_MEAN | mg.MGFR_WARM_START)
    u2, hist2, st2 = mg.mg_fr_solve(ctx, dev(rho), p, o2, u=u_d.clone())
    assert st2 == mg.MGFR_OK and len(hist2) == 1


@pytest.mark.parametrize("N,cn", [(4, 4), (2, 2), (8, 2)])
def test_degenerate_hierarchies(mg, ctx, N, cn):
    """N = coarsest_n: the whole solve is the coarsest-level smoother; N = 8 down to 2^3."""
    say(f"[solve] degenerate N={N} coarsest={cn}")
    p, m = both(8.0, 1e-5)
    rho = inputs.lognormal(N, 0.5, -2.0, seed=7) if N > 2 else np.array([1.3, 0.7] * 4).reshape(2, 2, 2)
    o = mg.mgfr_default_opts(tol=1e-12, coarsest_n=cn, coarsest_sweeps=2000, coarsest_rtol=1e-6)
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, o)
    assert st == mg.MGFR_OK, ctx.last_error()
    u_ref, _, st_ref = O.solve(rho, m, O.Opts(tol=1e-12, coarsest_n=cn, coarsest_sweeps=2000, coarsest_rtol=1e-6))
    assert st_ref == 0
    assert rel_err(u_d.cpu().numpy(), u_ref) <= 1e-10


def test_error_paths(mg, ctx):
    say("[solve] error paths")
    import torch
    p, _ = both(64.0, 1e-5)
    N = 16
    rho = inputs.small_box(N, 0)
    bad = rho.copy()
    bad[3, 4, 5] = np.nan
    _, _, st = mg.mg_fr_solve(ctx, dev(bad), p, raise_on_error=False)
    assert st == mg.MGFR_ENONFINITE
    _, _, st = mg.mg_fr_solve(ctx, dev(np.ones((12, 12, 12))), p, raise_on_error=False)
    assert st == mg.MGFR_EINVAL
    _, _, st = mg.mg_fr_solve(ctx, dev(rho), p, mg.mgfr_default_opts(coarsest_n=3), raise_on_error=False)
    assert st == mg.MGFR_EINVAL
    u = torch.zeros((N, N, N), dtype=torch.float64, device="cuda:0")
    u, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, mg.mgfr_default_opts(tol=1e-14, max_cycles=1), u=u,
                                 raise_on_error=False)
    assert st == mg.MGFR_ENOTCONV and len(hist) == 2 and hist[1] < hist[0]
    assert torch.isfinite(u).all() and (u != 0).all()


def _sampled_residual(u, rho, m, nsample, seed):
    N = u.shape[0]
    idx = np.random.default_rng(seed).choice(N ** 3, size=nsample, replace=False)
    return O.operator_at(u, m, 1.0 / N, idx, rho=rho)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,N,box,fr0", [("tophat-256-F5", 256, 256.0, 1e-5),
                                           ("halo-512-F6", 512, 512.0, 1e-6)])
def test_full_size_solution_satisfies_oracle_operator(mg, ctx, name, N, box, fr0, precision):
    """At the benchmark sizes the oracle's operator, evaluated on the GPU solution at sampled
    cells, is consistent with the reported rms residual <= 1e-8 (the residual is a property
    of the solution alone, so this holds whatever path produced it)."""
    say(f"[full] {name}: generating input")
    rho = inputs.tophat_box(N) if N == 256 else inputs.halo_box(N)
    p, m = both(box, fr0)
    say(f"[full] {name} {precision}: solving")
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    u_d, hist, st = mg.mg_fr_solve(ctx, dev(rho), p, mg.mgfr_default_opts(tol=1e-8, max_cycles=100, precision=prec))
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    u = u_d.cpu().numpy()
    say(f"[full] {name}: cycles={len(hist) - 1} final={hist[-1]:.3e}; oracle check")
    L = _sampled_residual(u, rho, m, 200000, seed=N)
    rms = np.sqrt(np.mean(L ** 2))
    assert rms <= 3e-8, rms
    # the GPU's own residual field agrees with the oracle's at the sampled cells
    d = mg.mgfr_residual(ctx, dev(rho), u_d, p).cpu().numpy().ravel()
    idx = np.random.default_rng(N).choice(N ** 3, size=200000, replace=False)
    assert np.abs(d[idx] - L).max() <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_maximum_size_sine_matches_one_dimensional_newton(mg, ctx, precision):
    """N = 1024, the largest grid the library takes (32-bit in-plane offsets, the most planes
    per workgroup): the x-only sine density of Sec. VI.A.3.  The 3-D solution must equal the
    brute-force 1-D Newton solution of the same discrete equations (paper_refs.newton_1d) in
    every cell.  The density is built on the device from the 1-D profile."""
    import paper_refs as P
    import torch
    N, box, fr0 = 1024, 256.0, 1e-5
    p, m = both(box, fr0)
    x = (np.arange(N) + 0.5) / N
    rho1 = 1.0 + P.sine_density(m, x)
    say(f"[max] N={N} {precision}: 1-D Newton reference")
    u1 = P.newton_1d(m, rho1, 1.0 / N, P.sine_u(m, x))
    rho = dev(rho1)[:, None, None].expand(N, N, N).contiguous()
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    say(f"[max] N={N} {precision}: solving")
    u_d, hist, st = mg.mg_fr_solve(ctx, rho, p, mg.mgfr_default_opts(tol=1e-11, max_cycles=100, precision=prec))
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    del rho
    err = (u_d - dev(u1)[:, None, None]).abs().max().item()
    say(f"[max] cycles={len(hist) - 1} final={hist[-1]:.2e} max|u - u_1d|={err:.2e}")
    assert err <= 1e-10  # |u| ~ 11: 1e-11 relative (measured 4.6e-12 FP64, 1.8e-13 mixed)
    del u_d
    torch.cuda.empty_cache()
