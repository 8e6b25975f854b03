"""Parity of the batched solves (refinement patches, independent boxes) against the oracle
(needs an MI355X).  Patches: both sides start from the same domain solution, so the
comparison is of the patch solves (boundary set-up, BC-modified operator, V-cycles).
Bar: double precision max|u - u*|/max|u*| <= 1e-10 per unit, both converged to
rms(L) <= 1e-10; mixed precision (single-precision correction V-cycles in the
double-precision defect-correction loop) <= 1e-6 at rms(L) <= 1e-8."""
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


def rel_err(u, ref):
    return np.abs(u - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("N0,thr,sizes", [(32, (3.0, 8.0), (8, 4)), (64, (10.0, 40.0, 150.0), (16, 8, 4))])
def test_patches_match_oracle(mg, ctx, N0, thr, sizes):
    say(f"[patches] N0={N0}")
    box, fr0 = 2.0 * N0, 1e-5
    rho0, patches, rho_packed = inputs.amr_workload(N0, seed=3, thresholds=thr, sizes=sizes)
    assert len(patches) >= 4 and max(p["level"] for p in patches) >= 2
    params = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    model = O.Model(box_mpc_h=box, fr0_abs=fr0)
    ud, hist, st = mg.mg_fr_solve(ctx, dev(rho0), params, mg.mgfr_default_opts(tol=1e-12))
    assert st == mg.MGFR_OK
    u_dom = ud.cpu().numpy()
    opts = mg.mgfr_default_opts(tol=1e-10)
    up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    up = up.cpu().numpy()
    rho_list = [rho_packed[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3) for p in patches]
    us, hs, sts = O.solve_patches(u_dom, patches, rho_list, model, O.Opts(tol=1e-10))
    for i, p in enumerate(patches):
        assert sts[i] == 0
        g = up[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3)
        assert rel_err(g, us[i]) <= 1e-10, (i, p)
        assert hists[i][-1] <= 1e-10


def test_patch_layout_errors(mg, ctx):
    say("[patches] layout errors")
    import torch
    N0 = 16
    params = mg.Params(box_mpc_h=32.0)
    ud = torch.zeros((N0, N0, N0), dtype=torch.float64, device="cuda:0") - 11.5
    rho = torch.ones(8 ** 3 * 2, dtype=torch.float64, device="cuda:0")
    good = dict(level=1, parent=-1, origin=(4, 4, 4), n=8, offset=0)
    cases = [
        [good, dict(good, origin=(6, 6, 6), offset=512)],                       # overlap
        [dict(good, origin=(3, 4, 4))],                                          # odd origin
        [dict(good, offset=600)],                                                # past the packed arrays
        [good, dict(level=2, parent=0, origin=(8, 8, 8), n=8, offset=512)],      # no margin in parent
        [dict(good, parent=0)],                                                  # level 1 with a patch parent
    ]
    for ps in cases:
        _, _, st = mg.mg_fr_solve_patches(ctx, ud, ps, rho, params, raise_on_error=False)
        assert st == mg.MGFR_EINVAL, ps
    # no patches: nothing to do
    _, _, st = mg.mg_fr_solve_patches(ctx, ud, [], rho, params, raise_on_error=False)
    assert st == mg.MGFR_OK
    # the truncation-error stop rule belongs to the domain solve
    _, _, st = mg.mg_fr_solve_patches(ctx, ud, [good], rho, params, mg.mgfr_default_opts(tau_alpha=0.3),
                                      raise_on_error=False)
    assert st == mg.MGFR_EINVAL


def test_batch_of_boxes_matches_oracle(mg, ctx):
    say("[batch] boxes")
    rng = np.random.default_rng(5)
    specs = []
    for b, N in enumerate([16, 32, 16, 32, 8, 64]):
        fr0 = 10.0 ** rng.uniform(-6, -4)
        sigma = rng.uniform(1.0, 2.0)
        specs.append((N, float(N), fr0, inputs.lognormal(N, sigma, -1.5, seed=b)))
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, mg.mgfr_default_opts(tol=1e-10))
    assert st == mg.MGFR_OK, ctx.last_error()
    for (N, box, fr0, rho), u, h in zip(specs, us, hists):
        ref, _, st_ref = O.solve(rho, O.Model(box_mpc_h=box, fr0_abs=fr0), O.Opts(tol=1e-10))
        assert st_ref == 0
        assert rel_err(u.cpu().numpy(), ref) <= 1e-10
        assert h[-1] <= 1e-10
    # one box alone gives the same field as in the batch (units are independent)
    u1, h1, st1 = mg.mg_fr_solve_batch(ctx, rhos[1:2], params[1:2], mg.mgfr_default_opts(tol=1e-10))
    assert st1 == mg.MGFR_OK
    assert np.array_equal(u1[0].cpu().numpy(), us[1].cpu().numpy())


@pytest.mark.parametrize("N0,thr,sizes", [(32, (3.0, 8.0), (8, 4)), (64, (10.0, 40.0, 150.0), (16, 8, 4))])
@pytest.mark.parametrize("inner", [1, 2])
def test_mixed_patches_match_oracle(mg, ctx, N0, thr, sizes, inner):
    say(f"[patches mixed] N0={N0} inner={inner}")
    box, fr0 = 2.0 * N0, 1e-5
    rho0, patches, rho_packed = inputs.amr_workload(N0, seed=3, thresholds=thr, sizes=sizes)
    params = mg.Params(box_mpc_h=box, fr0_abs=fr0)
    model = O.Model(box_mpc_h=box, fr0_abs=fr0)
    ud, hist, st = mg.mg_fr_solve(ctx, dev(rho0), params, mg.mgfr_default_opts(tol=1e-12))
    assert st == mg.MGFR_OK
    u_dom = ud.cpu().numpy()
    opts = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED, inner_cycles=inner)
    up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    up = up.cpu().numpy()
    rho_list = [rho_packed[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3) for p in patches]
    us, hs, sts = O.solve_patches(u_dom, patches, rho_list, model, O.Opts(tol=1e-11))
    for i, p in enumerate(patches):
        assert sts[i] == 0
        g = up[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3)
        assert rel_err(g, us[i]) <= 1e-6, (i, p, rel_err(g, us[i]))
        h = np.asarray(hists[i])
        assert h[-1] <= 1e-8
        assert np.all(np.diff(h) < 0), (i, h)


def test_mixed_batch_of_boxes_matches_oracle(mg, ctx):
    say("[batch mixed] boxes")
    rng = np.random.default_rng(5)
    specs = []
    for b, N in enumerate([16, 32, 16, 32, 8, 64]):
        fr0 = 10.0 ** rng.uniform(-6, -4)
        sigma = rng.uniform(1.0, 2.0)
        specs.append((N, float(N), fr0, inputs.lognormal(N, sigma, -1.5, seed=b)))
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    opts = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED)
    us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    for (N, box, fr0, rho), u, h in zip(specs, us, hists):
        # reference at 1e-10 (some of these boxes have their double-precision floor above 1e-12)
        ref, _, st_ref = O.solve(rho, O.Model(box_mpc_h=box, fr0_abs=fr0), O.Opts(tol=1e-10))
        assert st_ref == 0
        assert rel_err(u.cpu().numpy(), ref) <= 1e-6
        assert h[-1] <= 1e-8
    # a single box alone gives the same field as in the batch
    u1, h1, st1 = mg.mg_fr_solve_batch(ctx, rhos[1:2], params[1:2], opts)
    assert st1 == mg.MGFR_OK
    assert np.array_equal(u1[0].cpu().numpy(), us[1].cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(mg, ctx, precision):
    """With MGFR_GRAPH the launches of one cycle are captured once and replayed for every
    later cycle, with the norms, their host copy and the active-flag upload run eagerly in
    between.  Every replay must give what the eager launches give: the per-cycle residual
    histories and the final fields are compared bit for bit."""
    say(f"[graph] {precision}")
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    tol = 1e-8 if precision == "mixed" else 1e-10
    rng = np.random.default_rng(7)
    specs = []
    for b, N in enumerate([32, 16, 64, 32]):
        specs.append((N, float(N), 10.0 ** rng.uniform(-6, -4), inputs.lognormal(N, rng.uniform(1.0, 2.0), -1.5, seed=20 + b)))
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    out = {}
    for flags in (0, mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=flags)
        us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
        assert st == mg.MGFR_OK, ctx.last_error()
        out[flags] = ([u.cpu().numpy() for u in us], [np.asarray(h) for h in hists])
        if flags == mg.MGFR_PROFILE:
            check_profile(mg, ctx, opts)
    assert max(len(h) for h in out[0][1]) >= 4          # several replays
    for f in (mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        for a, b in zip(out[0][0], out[f][0]):
            assert np.array_equal(a, b)
        for a, b in zip(out[0][1], out[f][1]):
            assert np.array_equal(a, b)
    # patches (ghost faces, units of several depths) under a graph
    N0 = 32
    rho0, patches, rho_packed = inputs.amr_workload(N0, seed=3, thresholds=(3.0, 8.0), sizes=(8, 4))
    p = mg.Params(box_mpc_h=2.0 * N0, fr0_abs=1e-5)
    ud, _, st = mg.mg_fr_solve(ctx, dev(rho0), p, mg.mgfr_default_opts(tol=1e-12))
    assert st == mg.MGFR_OK
    res = {}
    for flags in (0, mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=flags)
        up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), p, opts)
        assert st == mg.MGFR_OK, ctx.last_error()
        res[flags] = (up.cpu().numpy(), [np.asarray(h) for h in hists])
        if flags == mg.MGFR_PROFILE:
            check_profile(mg, ctx, opts)
    for f in (mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        assert np.array_equal(res[0][0], res[f][0])
        for a, b in zip(res[0][1], res[f][1]):
            assert np.array_equal(a, b)


def check_profile(mg, ctx, opts):
    """MGFR_PROFILE on a batched solve: both colour launches of every finest-level sweep are
    timed (every V-cycle of a run whose units have more than one level), and the bytes
    credited are 24 (FP64) or 16 (single-precision correction) per finest-level cell update of
    the active units."""
    s = mg.mgfr_get_stats(ctx)
    mixed = opts.precision == mg.MGFR_MIXED
    vcycles = s["inner_cycles"] if mixed else s["cycles"]
    per = 2 * (opts.pre + opts.post)
    assert 0 < s["sweep_launches"] <= per * vcycles and s["sweep_launches"] % per == 0, s
    assert s["sweep_ms"] > 0.0
    assert s["sweep_bytes"] == (16 if mixed else 24) * s["finest_updates"], s
