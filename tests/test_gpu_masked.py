"""Parity of the GPU refinement-level solve with the mask scheme (mg_fr_solve_masked) with the
oracle's (oracle.solve_masked), on an MI355X.

Inputs are seeded and synthetic: a lognormal or halo density, a mask built the way an
oct-based AMR code refines (inputs.oct_mask: octs under dense coarse cells plus a one-oct
buffer), or a random fractional mask, and fixed values u_bar + a smooth Gaussian field.
Both sides run the same FAS V-cycles, so besides the solution (max |u - u*| <= 1e-9 with both
solved to an rms residual of 1e-11 over the active cells) the residual histories must agree
cycle by cycle (relative 1e-6 while above the rounding floor): that checks the coarse-level
rules (fractional restricted masks, masked restriction and prolongation) as well as the fine
equations.  Masked cells must come back bit-for-bit unchanged.
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


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0", dtype=dtype or torch.float64)


def oct_case(N, seed, frac=0.1, box=None, fr0=1e-5):
    rho = inputs.small_box(N, seed) if N <= 64 else inputs.tophat_box(N, seed, count=N // 4)
    od = rho.reshape(N // 2, 2, N // 2, 2, N // 2, 2).mean(axis=(1, 3, 5))
    mask = inputs.oct_mask(rho, float(np.quantile(od, 1.0 - frac)), expand=1)
    box = box or float(N)
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    u0 = O.constants(m, N)["ubar"] + 0.5 * inputs.gaussian_field(N, 1.0, -2.0, seed=seed + 40)
    return rho, mask, u0, box, fr0


def run_both(mg, ctx, rho, mask, u0, box, fr0, tol=1e-11, **kw):
    import torch
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    ur, hr, sr = O.solve_masked(rho, mask, m, u0, O.Opts(tol=tol, **kw))
    assert sr == 0, hr
    mask32 = mask.astype(np.float32)
    assert np.array_equal(mask32.astype(np.float64), mask)
    ud = dev(u0)
    ud, hg, sg = mg.mg_fr_solve_masked(ctx, dev(rho), dev(mask32, torch.float32), ud, p,
                                       mg.mgfr_default_opts(tol=tol, **kw))
    assert sg == mg.MGFR_OK, ctx.last_error()
    return ur, hr, ud.cpu().numpy(), hg


def check(ur, hr, ug, hg, mask, u0, bar=1e-9):
    err = np.abs(ug - ur).max()
    assert np.array_equal(ug[mask <= 0], u0[mask <= 0])
    assert err <= bar, err
    assert abs(len(hg) - len(hr)) <= 1
    k = min(len(hg), len(hr))
    above = hr[:k] > 1e-8 * hr[0]
    rel = np.abs(hg[:k] - hr[:k]) / hr[:k]
    assert np.all(rel[above] <= 1e-6), (hg, hr)
    return err


@pytest.mark.parametrize("N,seed,frac", [(16, 1, 0.2), (32, 0, 0.1), (64, 2, 0.1), (128, 1, 0.05)])
def test_oct_mask_matches_oracle(mg, ctx, N, seed, frac):
    say(f"[masked] oct mask N={N}")
    rho, mask, u0, box, fr0 = oct_case(N, seed, frac)
    ur, hr, ug, hg = run_both(mg, ctx, rho, mask, u0, box, fr0)
    err = check(ur, hr, ug, hg, mask, u0)
    say(f"  active {(mask > 0).mean():.3f}, cycles {len(hg) - 1}/{len(hr) - 1}, max err {err:.2e}")


@pytest.mark.parametrize("N,pre,post,planes", [(64, 2, 2, 0), (64, 1, 2, 4), (128, 2, 2, 0), (128, 2, 1, 8)])
def test_fused_sweep_matches_per_colour(mg, ctx, N, pre, post, planes):
    """A finest level of +1 / -1 masks (n >= 64) is swept both colours in one pass, out of place
    between the caller's u and a second buffer (tile = 0); tile = 1 keeps one launch per
    colour.  Every update sees the same operands in the same order, so fields and residual
    histories agree bit for bit, also with odd sweep counts (the field then ends in the second
    buffer and is copied back) and at several plane chunks."""
    import torch
    say(f"[masked] fused vs per colour N={N} pre={pre} post={post} planes={planes}")
    rho, mask, u0, box, fr0 = oct_case(N, 2, 0.1)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    out = []
    for tile in (1, 0):
        opts = mg.mgfr_default_opts(tol=1e-10, pre=pre, post=post, planes=planes, tile=tile)
        ud, hg, sg = mg.mg_fr_solve_masked(ctx, dev(rho), dev(mask.astype(np.float32), torch.float32), dev(u0), p,
                                           opts)
        assert sg == mg.MGFR_OK, ctx.last_error()
        out.append((ud.cpu().numpy(), np.asarray(hg)))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[1][0][mask <= 0], u0[mask <= 0])


def test_fractional_mask_matches_oracle(mg, ctx):
    """Mask values multiples of 1/4 in [-1, 1] on the finest level too (exact in float)."""
    say("[masked] fractional mask")
    N = 32
    rho, _, u0, box, fr0 = oct_case(N, 3)
    rng = np.random.default_rng(4)
    coarse = rng.integers(-4, 5, size=(N // 4,) * 3) / 4.0
    mask = np.repeat(np.repeat(np.repeat(coarse, 4, 0), 4, 1), 4, 2)
    assert (mask > 0).any() and (mask <= 0).any() and (mask == 0).any()
    ur, hr, ug, hg = run_both(mg, ctx, rho, mask, u0, box, fr0)
    err = check(ur, hr, ug, hg, mask, u0)
    say(f"  cycles {len(hg) - 1}, max err {err:.2e}")


def test_all_active_is_the_domain_solve(mg, ctx):
    say("[masked] all active")
    import torch
    N, box, fr0 = 64, 64.0, 1e-5
    rho = inputs.small_box(N, 5)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    ub = O.constants(O.Model(box_mpc_h=box, fr0_abs=fr0), N)["ubar"]
    o = mg.mgfr_default_opts(tol=1e-11)
    ud, hm, st = mg.mg_fr_solve_masked(ctx, dev(rho), torch.ones((N,) * 3, dtype=torch.float32, device="cuda:0"),
                                       dev(np.full((N,) * 3, ub)), p, o)
    assert st == mg.MGFR_OK
    uref, hd, st2 = mg.mg_fr_solve(ctx, dev(rho), p, o)
    assert st2 == mg.MGFR_OK
    assert (ud - uref).abs().max().item() <= 1e-10
    assert len(hm) == len(hd)


def test_cycle_settings(mg, ctx):
    """Other sweep counts and coarsest level: the same fixed point, and the same histories as
    the oracle with those settings."""
    say("[masked] settings")
    rho, mask, u0, box, fr0 = oct_case(32, 6, 0.15)
    ur, hr, ug, hg = run_both(mg, ctx, rho, mask, u0, box, fr0, pre=1, post=3, coarsest_n=2, max_step=0.5)
    check(ur, hr, ug, hg, mask, u0)
    ur2, hr2, ug2, hg2 = run_both(mg, ctx, rho, mask, u0, box, fr0, coarsest_n=8, coarsest_rtol=0.0,
                                  coarsest_sweeps=30)
    check(ur2, hr2, ug2, hg2, mask, u0)
    assert np.abs(ug - ug2).max() <= 1e-9


def test_subtract_mean_and_single_level(mg, ctx):
    """MGFR_SUBTRACT_MEAN (contrast about the mean density) against the oracle's
    subtract_mean, and a level that is its own coarsest level (8^3, coarsest_n 8: the whole
    solve runs in the one-workgroup kernel with the density as source)."""
    say("[masked] subtract mean, single level")
    import torch
    rho, mask, u0, box, fr0 = oct_case(32, 7, 0.15)
    rho = rho * 1.7  # mean 1.7: the two density references differ
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    ur, hr, sr = O.solve_masked(rho, mask, m, u0, O.Opts(tol=1e-11, subtract_mean=True))
    assert sr == 0
    ud, hg, sg = mg.mg_fr_solve_masked(ctx, dev(rho), dev(mask, torch.float32), dev(u0), p,
                                       mg.mgfr_default_opts(tol=1e-11, flags=mg.MGFR_SUBTRACT_MEAN))
    assert sg == mg.MGFR_OK, ctx.last_error()
    check(ur, hr, ud.cpu().numpy(), hg, mask, u0)
    N = 8
    rho8 = inputs.small_box(N, 2)
    mask8 = np.where(np.random.default_rng(3).random((N, N, N)) < 0.5, 1.0, -1.0)
    m8 = O.Model(box_mpc_h=16.0, fr0_abs=1e-5)
    u8 = O.constants(m8, N)["ubar"] + 0.3 * inputs.gaussian_field(N, 1.0, -2.0, seed=5)
    kw = dict(tol=1e-11, coarsest_n=8, coarsest_sweeps=400, max_cycles=40)
    ur8, hr8, sr8 = O.solve_masked(rho8, mask8, m8, u8, O.Opts(**kw))
    assert sr8 == 0, hr8
    ud8, hg8, sg8 = mg.mg_fr_solve_masked(ctx, dev(rho8), dev(mask8, torch.float32), dev(u8),
                                          mg.Params(box_mpc_h=16.0, fr0_abs=1e-5), mg.mgfr_default_opts(**kw))
    assert sg8 == mg.MGFR_OK, ctx.last_error()
    g8 = ud8.cpu().numpy()
    assert np.array_equal(g8[mask8 <= 0], u8[mask8 <= 0])
    assert np.abs(g8 - ur8).max() <= 1e-9


def test_masked_errors(mg, ctx):
    say("[masked] errors")
    import torch
    N = 16
    rho, mask, u0, box, fr0 = oct_case(N, 1, 0.2)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    m32 = dev(mask, torch.float32)
    bad = m32.clone()
    bad[1, 2, 3] = 1.5
    _, _, st = mg.mg_fr_solve_masked(ctx, dev(rho), bad, dev(u0), p, raise_on_error=False)
    assert st == mg.MGFR_EINVAL
    _, _, st = mg.mg_fr_solve_masked(ctx, dev(rho), m32, dev(u0), p, mg.mgfr_default_opts(precision=mg.MGFR_MIXED),
                                     raise_on_error=False)
    assert st == mg.MGFR_EINVAL
    r2 = rho.copy()
    r2[0, 0, 0] = np.nan
    _, _, st = mg.mg_fr_solve_masked(ctx, dev(r2), m32, dev(u0), p, raise_on_error=False)
    assert st == mg.MGFR_ENONFINITE
    # nothing active: no cycle, rms 0
    ud, h, st = mg.mg_fr_solve_masked(ctx, dev(rho), -torch.ones_like(m32), dev(u0), p)
    assert st == mg.MGFR_OK and len(h) == 1 and h[0] == 0.0
    assert np.array_equal(ud.cpu().numpy(), u0)


def test_masked_full_size(mg, ctx):
    """512^3 halo density with the oct mask of the densest quarter of octs (the configuration
    bench.py times), fixed values u_bar + a smooth field, tol 1e-8: masked cells unchanged,
    and the oracle's masked operator on the returned field gives the reported rms."""
    say("[masked] full size 512")
    import torch
    N, box, fr0 = 512, 512.0, 1e-6
    rho, mask = inputs.masked_level(N)
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    u0 = O.constants(m, N)["ubar"] + 0.5 * inputs.gaussian_field(N, 1.0, -2.0, seed=44)
    p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    ud, hg, st = mg.mg_fr_solve_masked(ctx, dev(rho), dev(mask, torch.float32), dev(u0), p,
                                       mg.mgfr_default_opts(tol=1e-8))
    assert st == mg.MGFR_OK, ctx.last_error()
    ug = ud.cpu().numpy()
    del ud
    act = mask > 0
    assert np.array_equal(ug[~act], u0[~act])
    L, _ = O.masked_operator(ug, u0, mask, m, rho=rho)
    rms = np.sqrt(np.mean(L[act] ** 2))
    say(f"  active {act.mean():.3f}, cycles {len(hg) - 1}, rms {hg[-1]:.3e}, oracle rms {rms:.3e}")
    assert rms <= 1e-8 * 1.001
    assert abs(rms - hg[-1]) <= 1e-3 * hg[-1]


def test_masked_maximum_size_all_active_sine(mg, ctx):
    """N = 1024, the largest grid the library takes, every cell active: the mask scheme
    reduces to the domain equations, so the x-only sine density of Sec. VI.A.3 must give the
    brute-force 1-D Newton solution of the discrete equations (paper_refs.newton_1d)."""
    import paper_refs as P
    import torch
    N, box, fr0 = 1024, 256.0, 1e-5
    m = O.Model(box_mpc_h=box, fr0_abs=fr0)
    x = (np.arange(N) + 0.5) / N
    rho1 = 1.0 + P.sine_density(m, x)
    say("[masked] max size: 1-D Newton reference")
    u1 = P.newton_1d(m, rho1, 1.0 / N, P.sine_u(m, x))
    rho = dev(rho1)[:, None, None].expand(N, N, N).contiguous()
    ones = torch.ones((N, N, N), dtype=torch.float32, device="cuda:0")
    u0 = torch.full_like(rho, O.constants(m, N)["ubar"])
    say("[masked] max size: solving")
    ud, hg, st = mg.mg_fr_solve_masked(ctx, rho, ones, u0, mg.Params(box_mpc_h=box, fr0_abs=fr0),
                                       mg.mgfr_default_opts(tol=1e-11, max_cycles=100))
    assert st == mg.MGFR_OK, (ctx.last_error(), hg)
    del rho, ones
    err = (ud - dev(u1)[:, None, None]).abs().max().item()
    say(f"  cycles {len(hg) - 1}, final {hg[-1]:.2e}, max|u - u_1d| {err:.2e}")
    assert err <= 1e-10
    del ud, u0
    torch.cuda.empty_cache()
