"""Parity of the batched solves (refinement patches, independent boxes) against the oracle
(needs an MI355X).  Patches: both sides start from the same domain solution, so the
comparison is of the patch solves (boundary set-up, BC-modified operator, V-cycles).
Bar: max|u - u*|/max|u*| <= 1e-10 per unit, both converged to rms(L) <= 1e-10."""
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
