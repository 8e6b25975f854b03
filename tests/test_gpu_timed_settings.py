"""Parity at the settings the benchmark times (needs an MI355X).

The benchmark autotunes the 512^3 solves (sweeps, single-precision V-cycles per outer
iteration, planes per workgroup and tile of the finest fused sweeps) and times what it picks.
These tests run those kernels at every setting the autotuner can choose:
- the double-precision fused red-black sweep (both tiles) against the two-pass (one kernel
  per colour) sweep, bit for bit, at 256^3 and 512^3 for 8 ... 128 planes per workgroup;
- the single-precision fused correction sweep (every tile) against its per-colour sweep at the
  same sizes and planes: bit for bit for the tiles with one column pair per thread, within a
  few units in the last place for the one that recovers b = exp(ub) as B - M;
- the 256^3 top-hat workload (box 256 Mpc/h, |f_R0| = 1e-5), every cell against the oracle's
  solution, for the double-precision solver at every planes setting and tile and the mixed
  solver at every planes setting with 1 and 2 single-precision V-cycles per outer iteration
  and at every tile;
- the 512^3 halo workload at the benchmark's settings, checked through the oracle's operator
  at sampled cells;
- the autotuner itself on a 128^3 problem: the options it returns converge and their solution
  matches the oracle.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1110_1379_amd import inputs

pytestmark = pytest.mark.gpu

PLANES = (8, 16, 32, 64, 128)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mg():
    import torch
    from paper_1110_1379_amd import mgfr
    assert torch.cuda.is_available(), "GPU tests need a GPU"
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


def both(box, fr0):
    from paper_1110_1379_amd import mgfr
    return mgfr.Params(box_mpc_h=box, fr0_abs=fr0), O.Model(box_mpc_h=box, fr0_abs=fr0)


def device_inputs(N, ubar, seed):
    """Seeded test fields made on the device: a lognormal density of mean 1 and a start
    field of the background plus noise."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    rho = torch.exp(0.8 * torch.randn((N, N, N), generator=g, device="cuda:0", dtype=torch.float64))
    rho /= rho.mean()
    u0 = ubar + 0.2 * torch.randn((N, N, N), generator=g, device="cuda:0", dtype=torch.float64)
    return rho, u0


@pytest.mark.parametrize("N", [256, 512])
def test_fp64_fused_sweep_is_bitwise_two_pass_at_every_planes_setting(mg, ctx, N):
    """Both tiles of the double-precision fused sweep (16 x 64 and 8 x 64) at every planes
    setting give the bits of the two-pass sweep."""
    import torch
    p, m = both(float(N), 1e-6)
    rho, u0 = device_inputs(N, O.constants(m, N)["ubar"], seed=N)
    say(f"[timed] FP64 two-pass reference N={N}")
    ref = mg.mgfr_smooth(ctx, rho, u0.clone(), p, nsweeps=3, variant=1)
    for tile in (1, 2):
        for planes in PLANES:
            say(f"[timed] FP64 fused N={N} tile={tile} planes={planes}")
            o = mg.mgfr_default_opts(planes=planes, tile=tile)
            got = mg.mgfr_smooth(ctx, rho, u0.clone(), p, nsweeps=3, variant=2, opts=o)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (N, tile, planes, (got - ref).abs().max().item())
    del rho, u0, ref, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N", [256, 512])
def test_fp32_fused_sweep_matches_per_colour_at_every_planes_setting(mg, ctx, N):
    """Tiles 1-3 and 5 (one tile column pair per thread; an updated cell's (B, M) formed again from
    (ub, e) as the per-colour kernel forms them): the bits of the per-colour sweep.  Tile 4
    (pairs over the halo) recovers b = exp(ub) of an updated cell as B - M instead, a
    difference of a few single-precision ulps in b and so in every later step: after 3 sweeps
    within 1e-5 of the largest change of e plus 4 ulps of e."""
    import torch
    p, m = both(float(N), 1e-6)
    ubar = O.constants(m, N)["ubar"]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(1000 + N)
    shape = (N, N, N)
    ub = (ubar + 0.2 * torch.randn(shape, generator=g, device="cuda:0")).float().contiguous()
    e0 = 1e-3 * torch.randn(shape, generator=g, device="cuda:0")
    big = torch.rand(shape, generator=g, device="cuda:0") < 0.05
    e0 = torch.where(big, 0.3 * torch.randn(shape, generator=g, device="cuda:0"), e0).float().contiguous()
    f = (0.05 * torch.randn(shape, generator=g, device="cuda:0")).float().contiguous()
    say(f"[timed] FP32 per-colour reference N={N}")
    ref = mg.mgfr_smooth32(ctx, ub, e0.clone(), f, p, nsweeps=3, variant=1)
    change = (ref - e0).abs().max().item()
    assert change > 0.0
    bound = 1e-5 * change + 4 * 1.1920929e-7 * e0.abs().max().item()
    for tile in (1, 2, 3, 4, 5):
        for planes in PLANES:
            say(f"[timed] FP32 fused N={N} tile={tile} planes={planes}")
            o = mg.mgfr_default_opts(planes=planes, tile=tile)
            got = mg.mgfr_smooth32(ctx, ub, e0.clone(), f, p, nsweeps=3, variant=2, opts=o)
            torch.cuda.synchronize()
            if tile != 4:
                assert torch.equal(got, ref), (N, tile, planes, (got - ref).abs().max().item())
            else:
                d = (got - ref).abs().max().item()
                say(f"[timed]   max |fused - per-colour| = {d:.3e} (largest change {change:.3e}, bound {bound:.3e})")
                assert d <= bound, (N, planes, d, bound)
    del ub, e0, f, ref, got
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def tophat256(mg):
    N = 256
    say("[timed] tophat256: generating the density")
    rho = inputs.tophat_box(N)
    p, m = both(256.0, 1e-5)
    say(f"[timed] tophat256: oracle solve to 1e-12 on {O.threads()} host threads")
    u_ref, h_ref, st = O.solve(rho, m, O.Opts(tol=1e-12))
    assert st == 0, h_ref
    say(f"[timed] tophat256: oracle took {len(h_ref) - 1} cycles")
    return rho, p, u_ref, len(h_ref) - 1


def test_tophat256_fp64_every_cell_matches_oracle(mg, ctx, tophat256):
    """Double-precision solver at every planes setting and tile of its finest sweeps, both
    sides at rms(L) <= 1e-12: max|u - u*| / max|u*| <= 1e-10."""
    import torch
    rho, p, u_ref, ncyc = tophat256
    rho_d, ref_d = dev(rho), dev(u_ref)
    scale = ref_d.abs().max().item()
    for planes, tile in [(pl, 0) for pl in (0,) + PLANES] + [(64, 2), (128, 2)]:
        say(f"[timed] tophat256 FP64 planes={planes} tile={tile}")
        u, hist, st = mg.mg_fr_solve(ctx, rho_d, p, mg.mgfr_default_opts(tol=1e-12, planes=planes, tile=tile,
                                                                        max_cycles=100))
        assert st == mg.MGFR_OK, (ctx.last_error(), hist)
        err = (u - ref_d).abs().max().item() / scale
        say(f"[timed]   cycles={len(hist) - 1} (oracle {ncyc}) rel err {err:.2e}")
        assert err <= 1e-10
        assert abs((len(hist) - 1) - ncyc) <= 1
    del rho_d, ref_d, u
    torch.cuda.empty_cache()


def test_tophat256_mixed_every_cell_matches_oracle(mg, ctx, tophat256):
    """Mixed solver (single-precision V-cycles in the double-precision defect correction) at
    every planes setting with 1, 2 and 3 inner V-cycles, at rms(L) <= 1e-8: max|u - u*| / max|u*|
    <= 1e-6 against the oracle at 1e-12.  The outer iteration count is pinned too: a fault in
    the single-precision sweep would only slow the outer loop down, since the double-precision
    residual corrects whatever the inner cycles return.  With k inner V-cycles the outer loop
    must contract like k double-precision V-cycles: at most ceil(c / k) + 1 iterations, where c
    is the double-precision solver's cycle count to the same tolerance."""
    import math
    import torch
    rho, p, u_ref, _ = tophat256
    rho_d, ref_d = dev(rho), dev(u_ref)
    scale = ref_d.abs().max().item()
    _, h64, st = mg.mg_fr_solve(ctx, rho_d, p, mg.mgfr_default_opts(tol=1e-8, max_cycles=100))
    assert st == mg.MGFR_OK
    c64 = len(h64) - 1
    settings = [(inner, planes, 0) for inner in (1, 2, 3) for planes in (0,) + PLANES]
    settings += [(inner, planes, tile) for inner in (2, 3) for tile in (1, 2, 3, 4, 5) for planes in (32, 64)]
    for inner, planes, tile in settings:
        say(f"[timed] tophat256 mixed inner={inner} planes={planes} tile={tile}")
        o = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED, inner_cycles=inner, planes=planes,
                                 tile=tile, max_cycles=100)
        u, hist, st = mg.mg_fr_solve(ctx, rho_d, p, o)
        assert st == mg.MGFR_OK, (ctx.last_error(), hist)
        err = (u - ref_d).abs().max().item() / scale
        say(f"[timed]   outer={len(hist) - 1} (FP64 cycles {c64}) rel err {err:.2e}")
        assert err <= 1e-6
        assert len(hist) - 1 <= math.ceil(c64 / inner) + 1, (hist, c64)
    del rho_d, ref_d, u
    torch.cuda.empty_cache()


def _sampled_operator_check(mg, ctx, u_d, rho, rho_d, p, m, N, nsample=100000):
    u = u_d.cpu().numpy()
    idx = np.random.default_rng(N).choice(N ** 3, size=nsample, replace=False)
    L = O.operator_at(u, m, 1.0 / N, idx, rho=rho)
    d = mg.mgfr_residual(ctx, rho_d, u_d, p).cpu().numpy().ravel()[idx]
    return np.sqrt(np.mean(L ** 2)), np.abs(d - L).max()


@pytest.mark.parametrize("precision,inner,planes,tile", [("fp64", 1, 128, 0), ("fp64", 1, 64, 0), ("mixed", 2, 0, 0),
                                                         ("mixed", 2, 64, 3), ("mixed", 2, 128, 0), ("mixed", 1, 0, 0),
                                                         ("mixed", 3, 32, 3), ("mixed", 3, 64, 3)])
def test_halo512_at_benchmark_settings(mg, ctx, precision, inner, planes, tile):
    """The 512^3 halo workload solved at the settings the autotuner picks for the benchmark:
    the oracle's operator at 100 000 sampled cells of the GPU field gives rms <= 3e-8 (the
    solve stops at 1e-8) and the GPU's own residual agrees with it there."""
    import torch
    N = 512
    key = "halo512"
    if key not in _cache:
        say("[timed] halo512: generating the density")
        _cache[key] = inputs.halo_box(N)
    rho = _cache[key]
    p, m = both(512.0, 1e-6)
    rho_d = dev(rho)
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    say(f"[timed] halo512 {precision} inner={inner} planes={planes} tile={tile}")
    o = mg.mgfr_default_opts(tol=1e-8, precision=prec, inner_cycles=inner, planes=planes, tile=tile, max_cycles=100)
    u_d, hist, st = mg.mg_fr_solve(ctx, rho_d, p, o)
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    rms, agree = _sampled_operator_check(mg, ctx, u_d, rho, rho_d, p, m, N)
    say(f"[timed]   cycles={len(hist) - 1} final={hist[-1]:.2e} oracle rms at samples {rms:.2e}")
    assert rms <= 3e-8, rms
    assert agree <= 1e-10
    del rho_d, u_d
    torch.cuda.empty_cache()


_cache = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuner_options_converge_and_match_oracle(mg, ctx, precision):
    """mgfr_autotune on a 128^3 top-hat problem: the options it returns are among its
    candidates, converge, and their solution matches the oracle (FP64 at 1e-12: <= 1e-10
    relative; mixed at 1e-8: <= 1e-6)."""
    import torch
    N = 128
    rho = inputs.tophat_box(N, 1, count=25)
    p, m = both(128.0, 1e-5)
    rho_d = dev(rho)
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    base = mg.mgfr_default_opts(tol=1e-8, precision=prec, max_cycles=100)
    say(f"[timed] autotune 128^3 {precision}")
    best, ms = mg.mgfr_autotune(ctx, rho_d, p, base=base)
    tuned = {k: getattr(best, k) for k in mg.TUNED_FIELDS}
    say(f"[timed]   best {tuned} {ms:.2f} ms")
    assert ms > 0.0
    assert (best.pre, best.post) in {(1, 1), (2, 1), (1, 2), (2, 2), (3, 3)}
    assert best.planes in (0,) + PLANES
    assert best.tile in ((0, 1, 2, 3, 4, 5) if precision == "mixed" else (0, 1, 2))
    assert best.inner_cycles in ((1, 2, 3) if precision == "mixed" else (1,))
    assert best.tol == base.tol and best.precision == prec and best.max_cycles == base.max_cycles
    u_ref, _, st_ref = O.solve(rho, m, O.Opts(tol=1e-12))
    assert st_ref == 0
    if precision == "fp64":
        best.tol = 1e-12
    u, hist, st = mg.mg_fr_solve(ctx, rho_d, p, best)
    assert st == mg.MGFR_OK, (ctx.last_error(), hist)
    err = np.abs(u.cpu().numpy() - u_ref).max() / np.abs(u_ref).max()
    assert err <= (1e-10 if precision == "fp64" else 1e-6), err
    del rho_d, u
    torch.cuda.empty_cache()
