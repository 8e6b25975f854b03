"""Parity of the GPU TSC density assignment and force interpolation (mgfr_tsc_density,
mgfr_tsc_force) with the oracle (oracle/tsc.py), on an MI355X.

Particles come from the seeded clustered generator (inputs.particles); potentials from the
oracle's periodic Poisson solve of the oracle's own density, or a seeded smooth field.  The
density sums each cell's contributions in an order of its own (particles sorted by cell), so
it is compared to a bar of 1e-12 of its maximum and checked to repeat bit for bit; the force
evaluates the same products and sums in the same order as the oracle (no contraction), so it
is compared to 1e-13 of the largest term and reported when bit-identical.  At 512^3 particles on the 512^3 grid (the configuration bench.py times) the
density is checked at sampled cells against the brute-force sum over the particles near
them, the total mass exactly, and the force at sampled particles.
"""
import sys

import numpy as np
import pytest

from oracle import poisson as P
from oracle import tsc
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


@pytest.mark.parametrize("Ng,N", [(2, 4), (16, 32), (32, 32), (64, 64), (64, 128)])
def test_density_and_force_match_oracle(mg, ctx, Ng, N):
    say(f"[tsc] {Ng}^3 particles on {N}^3")
    pos = inputs.particles(Ng, seed=Ng + N)
    m = N ** 3 / len(pos)
    ref = tsc.deposit(pos, N, m)
    pd = dev(pos)
    rho = mg.mgfr_tsc_density(ctx, pd, N, m).cpu().numpy()
    # a fixed summation order: the same bits on a second call
    assert np.array_equal(rho, mg.mgfr_tsc_density(ctx, pd, N, m).cpu().numpy())
    err = np.abs(rho - ref).max()
    assert err <= 1e-12 * ref.max(), err
    assert abs(rho.sum() - len(pos) * m) <= 1e-12 * len(pos) * m
    phi = P.solve(ref - 1.0)
    F = tsc.force(phi, pos)
    G = mg.mgfr_tsc_force(ctx, dev(phi), pd).cpu().numpy()
    scale = N * np.abs(phi).max()
    ferr = np.abs(G - F).max()
    say(f"  density max err {err:.2e} (max {ref.max():.1f}), force max err {ferr:.2e}, "
        f"bit-identical {np.array_equal(G, F)}")
    assert ferr <= 1e-13 * scale


@pytest.mark.parametrize("N", [512, 1024])
def test_density_rows_of_several_segments(mg, ctx, N):
    """N = 512 and 1024 (the largest grid): each row is split over two or four workgroups, so
    the wrapped source cells at both row ends, the segment seams and segments with neither
    end are exercised; every cell is compared to the oracle."""
    say(f"[tsc] 64^3 particles on {N}^3")
    pos = inputs.particles(64, seed=17)
    m = N ** 3 / len(pos)
    ref = tsc.deposit(pos, N, m)
    rho = mg.mgfr_tsc_density(ctx, dev(pos), N, m).cpu().numpy()
    err = np.abs(rho - ref).max()
    say(f"  density max err {err:.2e} (max {ref.max():.1f})")
    assert err <= 1e-12 * ref.max()


def test_gpu_pair_conserves_momentum(mg, ctx):
    """GPU density -> GPU Poisson solve (background scalaron) -> GPU forces: the total force
    vanishes (the TSC pair is momentum conserving; the Poisson operator is symmetric)."""
    say("[tsc] momentum")
    import torch
    Ng, N, box = 64, 64, 64.0
    pos = dev(inputs.particles(Ng, seed=9))
    rho = mg.mgfr_tsc_density(ctx, pos, N, N ** 3 / Ng ** 3)
    params = mg.Params(box_mpc_h=box, fr0_abs=1e-5)
    ub = mg.mgfr_constants(params, N)["ubar"]
    u = torch.full_like(rho, ub)
    phi, hist, st = mg.mg_poisson_solve(ctx, rho, u, params, mg.mgfr_default_opts(tol=1e-13, max_cycles=80))
    assert st == mg.MGFR_OK, ctx.last_error()
    F = mg.mgfr_tsc_force(ctx, phi, pos)
    tot = F.sum(dim=0).abs().cpu().numpy()
    scale = F.abs().sum(dim=0).cpu().numpy()
    say(f"  |sum F| / sum |F| = {(tot / scale).max():.2e}")
    assert np.all(tot <= 1e-10 * scale)


def test_tsc_errors(mg, ctx):
    say("[tsc] errors")
    import torch
    pos = dev(np.array([[0.1, 0.2, np.nan]]))
    with pytest.raises(mg.MgfrError):
        mg.mgfr_tsc_density(ctx, pos, 16, 1.0)
    with pytest.raises(mg.MgfrError):
        mg.mgfr_tsc_density(ctx, dev(np.zeros((4, 3))), 12, 1.0)
    # no particles: an empty density; positions exactly at 1.0 wrap to 0
    rho = mg.mgfr_tsc_density(ctx, torch.empty((0, 3), dtype=torch.float64, device="cuda:0"), 16, 1.0)
    assert rho.abs().max().item() == 0.0
    p1 = np.array([[1.0, 0.5, 0.999999999999]])
    assert np.array_equal(mg.mgfr_tsc_density(ctx, dev(p1), 16, 1.0).cpu().numpy(), tsc.deposit(p1, 16))


def test_tsc_full_size(mg, ctx):
    say("[tsc] full size 512")
    N = Ng = 512
    pos = inputs.particles(Ng, seed=3)
    pd = dev(pos)
    rho = mg.mgfr_tsc_density(ctx, pd, N, 1.0).cpu().numpy()
    assert abs(rho.mean() - 1.0) <= 1e-12
    # sampled cells: brute-force sums over the particles whose nearest cell is within one cell
    s = np.mod(pos * N, N)
    near = np.floor(s).astype(np.int64) % N
    key = (near[:, 0] * N + near[:, 1]) * N + near[:, 2]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    rng = np.random.default_rng(1)
    cells = rng.integers(0, N, size=(48, 3))
    cells[:8] = np.array(np.unravel_index(np.argsort(rho, axis=None)[-8:], rho.shape)).T  # densest
    worst = 0.0
    for c in cells:
        sel = []
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for z in (-1, 0, 1):
                    k = (((c[0] + a) % N) * N + (c[1] + b) % N) * N + (c[2] + z) % N
                    lo, hi = np.searchsorted(skey, k), np.searchsorted(skey, k, side="right")
                    sel.append(order[lo:hi])
        sel = np.concatenate(sel)
        val = tsc.deposit(pos[sel], N)[c[0], c[1], c[2]] if len(sel) else 0.0
        worst = max(worst, abs(val - rho[c[0], c[1], c[2]]) / max(1.0, abs(val)))
    say(f"  mean {rho.mean():.15f}, max {rho.max():.1f}, sampled worst rel err {worst:.2e}")
    assert worst <= 1e-12
    # force at sampled particles from a smooth potential
    phi = inputs.gaussian_field(N, 1.0, -3.0, seed=21)
    G = mg.mgfr_tsc_force(ctx, dev(phi), pd).cpu().numpy()
    idx = rng.integers(0, len(pos), 4096)
    F = tsc.force(phi, pos[idx])
    ferr = np.abs(G[idx] - F).max()
    say(f"  sampled force max err {ferr:.2e}, bit-identical {np.array_equal(G[idx], F)}")
    assert ferr <= 1e-13 * N * np.abs(phi).max()
