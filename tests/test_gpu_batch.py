"""Parity of the batched solves (refinement patches, independent boxes) against the oracle
(needs an MI355X).  Patches: both sides start from the same domain solution, so the
comparison is of the patch solves (boundary set-up, BC-modified operator, V-cycles).
Bar: double precision max|u - u*|/max|u*| <= 1e-10 per unit, both converged to
rms(L) <= 1e-10; mixed precision (single-precision correction V-cycles in the
double-precision defect-correction loop) <= 1e-6 at rms(L) <= 1e-8."""
import os
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


# the last case holds 64^3 patches (32 parent cells) on both levels, with 5-level hierarchies
PATCH_CASES = [(32, (3.0, 8.0), (8, 4)), (64, (10.0, 40.0, 150.0), (16, 8, 4)), (64, (3.0, 10.0), (32, 16, 8, 4))]

# (name, flags, unit_n): the default engine with units of side <= 16 solved whole by one
# workgroup (larger ones launched per phase on their fine levels and finished by one
# workgroup each below 16), the same with 8 and with 64 (every unit whole), and the per-phase
# engine with host stop tests
ENGINES = [("units16", 0, 0), ("units8", 0, 8), ("units64", 0, 64), ("phases", 16, 0)]

_patch_cache = {}


def patch_case(mg, ctx, N0, thr, sizes, tol):
    """Domain solution (GPU), patches and the oracle's patch solutions at tol, computed once."""
    key = (N0, thr, sizes, tol)
    if key not in _patch_cache:
        box, fr0 = 2.0 * N0, 1e-5
        rho0, patches, rho_packed = inputs.amr_workload(N0, seed=3, thresholds=thr, sizes=sizes)
        params = mg.Params(box_mpc_h=box, fr0_abs=fr0)
        model = O.Model(box_mpc_h=box, fr0_abs=fr0)
        ud, hist, st = mg.mg_fr_solve(ctx, dev(rho0), params, mg.mgfr_default_opts(tol=1e-12))
        assert st == mg.MGFR_OK
        rho_list = [rho_packed[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3) for p in patches]
        us, hs, sts = O.solve_patches(ud.cpu().numpy(), patches, rho_list, model, O.Opts(tol=tol))
        assert all(st == 0 for st in sts)
        _patch_cache[key] = (ud, patches, rho_packed, params, us)
    return _patch_cache[key]


@pytest.mark.parametrize("engine", ENGINES, ids=[e[0] for e in ENGINES])
@pytest.mark.parametrize("N0,thr,sizes", PATCH_CASES)
def test_patches_match_oracle(mg, ctx, N0, thr, sizes, engine):
    say(f"[patches] N0={N0} sizes={sizes} engine={engine[0]}")
    ud, patches, rho_packed, params, us = patch_case(mg, ctx, N0, thr, sizes, 1e-10)
    assert len(patches) >= 4 and max(p["level"] for p in patches) >= 2
    if max(sizes) == 32:
        assert {p["level"] for p in patches if p["n"] == 64} == {1, 2}
    opts = mg.mgfr_default_opts(tol=1e-10, flags=engine[1], unit_n=engine[2])
    up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    up = up.cpu().numpy()
    for i, p in enumerate(patches):
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


# up to 128^3, the largest box of the batch workload (6-level hierarchy)
BOX_SIDES = [16, 32, 16, 32, 8, 64, 128]


_box_cache = {}


def box_specs():
    rng = np.random.default_rng(5)
    specs = []
    for b, N in enumerate(BOX_SIDES):
        fr0 = 10.0 ** rng.uniform(-6, -4)
        sigma = rng.uniform(1.0, 2.0)
        specs.append((N, float(N), fr0, inputs.lognormal(N, sigma, -1.5, seed=b)))
    return specs


def box_refs(specs):
    """The oracle's solution of every box at 1e-10, computed once."""
    if "refs" not in _box_cache:
        refs = []
        for N, box, fr0, rho in specs:
            ref, _, st_ref = O.solve(rho, O.Model(box_mpc_h=box, fr0_abs=fr0), O.Opts(tol=1e-10))
            assert st_ref == 0
            refs.append(ref)
        _box_cache["refs"] = refs
    return _box_cache["refs"]


@pytest.mark.parametrize("engine", ENGINES, ids=[e[0] for e in ENGINES])
def test_batch_of_boxes_matches_oracle(mg, ctx, engine):
    say(f"[batch] boxes engine={engine[0]}")
    specs = box_specs()
    refs = box_refs(specs)
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    opts = mg.mgfr_default_opts(tol=1e-10, flags=engine[1], unit_n=engine[2])
    us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    for ref, u, h in zip(refs, us, hists):
        assert rel_err(u.cpu().numpy(), ref) <= 1e-10
        assert h[-1] <= 1e-10
    # one box alone gives the same field as in the batch (units are independent)
    u1, h1, st1 = mg.mg_fr_solve_batch(ctx, rhos[1:2], params[1:2], opts)
    assert st1 == mg.MGFR_OK
    assert np.array_equal(u1[0].cpu().numpy(), us[1].cpu().numpy())


@pytest.mark.parametrize("engine", ENGINES, ids=[e[0] for e in ENGINES])
@pytest.mark.parametrize("N0,thr,sizes", PATCH_CASES)
@pytest.mark.parametrize("inner", [1, 2])
def test_mixed_patches_match_oracle(mg, ctx, N0, thr, sizes, inner, engine):
    say(f"[patches mixed] N0={N0} sizes={sizes} inner={inner} engine={engine[0]}")
    ud, patches, rho_packed, params, us = patch_case(mg, ctx, N0, thr, sizes, 1e-11)
    opts = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED, inner_cycles=inner, flags=engine[1],
                                unit_n=engine[2])
    up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    up = up.cpu().numpy()
    for i, p in enumerate(patches):
        g = up[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3)
        assert rel_err(g, us[i]) <= 1e-6, (i, p, rel_err(g, us[i]))
        h = np.asarray(hists[i])
        assert h[-1] <= 1e-8
        assert np.all(np.diff(h) < 0), (i, h)


@pytest.mark.parametrize("engine", ENGINES, ids=[e[0] for e in ENGINES])
def test_mixed_batch_of_boxes_matches_oracle(mg, ctx, engine):
    say(f"[batch mixed] boxes engine={engine[0]}")
    specs = box_specs()
    # reference at 1e-10 (some of these boxes have their double-precision floor above 1e-12)
    refs = box_refs(specs)
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    opts = mg.mgfr_default_opts(tol=1e-8, precision=mg.MGFR_MIXED, flags=engine[1], unit_n=engine[2])
    us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    for ref, u, h in zip(refs, us, hists):
        assert rel_err(u.cpu().numpy(), ref) <= 1e-6
        assert h[-1] <= 1e-8
    # a single box alone gives the same field as in the batch
    u1, h1, st1 = mg.mg_fr_solve_batch(ctx, rhos[1:2], params[1:2], opts)
    assert st1 == mg.MGFR_OK
    assert np.array_equal(u1[0].cpu().numpy(), us[1].cpu().numpy())


# the settings the batch bench tries (and may time): (precision, pre, post, inner cycles)
TIMED_BATCH = [(prec, *cand) for prec, cands in (("fp64", [(2, 2, 1), (1, 1, 1), (2, 1, 1)]),
                                                  ("mixed", [(2, 2, 1), (2, 2, 2), (2, 2, 3)])) for cand in cands]


def test_timed_batch_settings_are_the_bench_candidates():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    assert sorted(TIMED_BATCH) == sorted((p, *c) for p, cs in bench.BATCH_CANDIDATES.items() for c in cs)


@pytest.mark.parametrize("precision,pre,post,inner", TIMED_BATCH, ids=["-".join(map(str, t)) for t in TIMED_BATCH])
def test_batch_at_the_timed_settings_matches_oracle(mg, ctx, precision, pre, post, inner):
    """Every setting the batch bench may time, in its engine (workgroup per unit), against the
    oracle's fields at 1e-10: double precision to <= 1e-10 at rms 1e-10, mixed to <= 1e-6 at
    rms 1e-8."""
    say(f"[batch timed settings] {precision} pre={pre} post={post} inner={inner}")
    specs = box_specs()
    refs = box_refs(specs)
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    fp64 = precision == "fp64"
    tol = 1e-10 if fp64 else 1e-8
    opts = mg.mgfr_default_opts(tol=tol, precision=mg.MGFR_FP64 if fp64 else mg.MGFR_MIXED, pre=pre, post=post,
                                inner_cycles=inner)
    us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
    assert st == mg.MGFR_OK, ctx.last_error()
    for ref, u, h in zip(refs, us, hists):
        assert rel_err(u.cpu().numpy(), ref) <= (1e-10 if fp64 else 1e-6)
        assert h[-1] <= tol


@pytest.mark.parametrize("engine", [e for e in ENGINES if e[0] in ("units16", "phases")], ids=["units16", "phases"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(mg, ctx, precision, engine):
    """With MGFR_GRAPH the launches of one cycle are captured once and replayed for every
    later cycle (default engine: with the device stop test inside the graph; per-phase engine:
    with the norms, their host copy and the active-flag upload run eagerly in between).  Every
    replay must give what the eager launches give: the per-cycle residual histories and the
    final fields are compared bit for bit.  MGFR_PROFILE (HIP events around the finest-level
    sweeps) must not change them either."""
    say(f"[graph] {precision} engine={engine[0]}")
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
        opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=flags | engine[1], unit_n=engine[2])
        us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
        assert st == mg.MGFR_OK, ctx.last_error()
        out[flags] = ([u.cpu().numpy() for u in us], [np.asarray(h) for h in hists])
        if flags == mg.MGFR_PROFILE:
            check_profile(mg, ctx, opts, [s[0] for s in specs], out[flags][1])
    assert max(len(h) for h in out[0][1]) >= 4          # several replays
    for f in (mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        for a, b in zip(out[0][0], out[f][0]):
            assert np.array_equal(a, b)
        for a, b in zip(out[0][1], out[f][1]):
            assert np.array_equal(a, b)
    # patches (ghost faces, units of several depths) under a graph
    N0 = 32
    rho0, patches, rho_packed = inputs.amr_workload(N0, seed=3, thresholds=(3.0, 8.0), sizes=(16, 8, 4))
    p = mg.Params(box_mpc_h=2.0 * N0, fr0_abs=1e-5)
    ud, _, st = mg.mg_fr_solve(ctx, dev(rho0), p, mg.mgfr_default_opts(tol=1e-12))
    assert st == mg.MGFR_OK
    res = {}
    for flags in (0, mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=flags | engine[1], unit_n=engine[2])
        up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), p, opts)
        assert st == mg.MGFR_OK, ctx.last_error()
        res[flags] = (up.cpu().numpy(), [np.asarray(h) for h in hists])
        if flags == mg.MGFR_PROFILE:
            check_profile(mg, ctx, opts, [q["n"] for q in patches], res[flags][1])
    for f in (mg.MGFR_GRAPH, mg.MGFR_PROFILE):
        assert np.array_equal(res[0][0], res[f][0])
        for a, b in zip(res[0][1], res[f][1]):
            assert np.array_equal(a, b)


def check_profile(mg, ctx, opts, sides, hists):
    """MGFR_PROFILE on a batched solve: the launches of the finest-level sweeps are timed (two
    per sweep and table of a depth, one per colour; two per pair of fused sweeps of periodic
    boxes in a mixed solve, so at least one per sweep), and the bytes credited are 24 (FP64) or 12
    (single-precision correction) per finest-level cell update.  Per-phase engine: every
    unit's finest level, the units active in each cycle.  Default engine: the finest levels of
    the units launched per phase (side above unit_n), every cycle each of them ran (the sweeps
    inside the one-workgroup kernels are not timed)."""
    s = mg.mgfr_get_stats(ctx)
    mixed = opts.precision == mg.MGFR_MIXED
    bpc = 12 if mixed else 24
    per_sweep = 2 * (opts.pre + opts.post)
    if opts.flags & mg.MGFR_PER_PHASE:
        vcycles = s["inner_cycles"] if mixed else s["cycles"]
        sweeps = (opts.pre + opts.post) * vcycles
        # up to three tables per depth: per cell, column tiles, fused pairs
        assert sweeps <= s["sweep_launches"] <= 3 * per_sweep * vcycles and s["sweep_launches"] % 2 == 0, s
        assert s["sweep_ms"] > 0.0
        assert s["sweep_bytes"] == bpc * s["finest_updates"], s
        return
    W = max(opts.unit_n or 16, opts.coarsest_n)
    inner = opts.inner_cycles if mixed else 1
    large = [(n, len(h) - 1) for n, h in zip(sides, hists) if n > W]
    assert s["sweep_bytes"] == bpc * sum(n ** 3 * k for n, k in large) * (opts.pre + opts.post) * inner, s
    if large:
        kmax = max(k for _, k in large)
        assert s["sweep_launches"] >= (opts.pre + opts.post) * inner * kmax and s["sweep_launches"] % 2 == 0, s
        assert s["sweep_ms"] > 0.0
    else:
        assert s["sweep_launches"] == 0, s


@pytest.mark.parametrize("engine", [e for e in ENGINES if e[0] in ("units16", "phases")], ids=["units16", "phases"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_column_sweep_matches_per_cell_sweep(mg, ctx, precision, engine):
    """The sweeps of unit levels of side >= 32 walk column tiles: by default (tile = 0) a mixed
    solve sweeps periodic boxes in pairs of fused two-colour sweeps and a double-precision one
    walks them one colour per launch, at depths with at least 256 tiles (per cell below);
    tile = 3 sweeps boxes and patches in fused pairs at every depth, and tile = 2 walks every
    level one colour per launch; with tile = 1 they run one thread per cell of the colour.
    All evaluate every cell update with the same operands in the same order, so fields and
    residual histories agree bit for bit: periodic boxes of sides 32 - 128 (also with odd
    sweep counts, where one sweep of a group runs in place), and patches of side 32 and 64
    (ghost faces)."""
    say(f"[column sweep] {precision} engine={engine[0]}")
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    tol = 1e-8 if precision == "mixed" else 1e-10
    rng = np.random.default_rng(9)
    specs = []
    for b, N in enumerate([32, 128, 64, 16]):
        specs.append((N, float(N), 10.0 ** rng.uniform(-6, -4), inputs.lognormal(N, rng.uniform(1.0, 2.0), -1.5, seed=40 + b)))
    rhos = [dev(s[3]) for s in specs]
    params = [mg.Params(box_mpc_h=s[1], fr0_abs=s[2]) for s in specs]
    for pre, post in ((2, 2), (1, 3)):
        out = []
        for tile in (1, 0, 2, 3):
            opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=engine[1], unit_n=engine[2], tile=tile,
                                        pre=pre, post=post)
            us, hists, st = mg.mg_fr_solve_batch(ctx, rhos, params, opts)
            assert st == mg.MGFR_OK, ctx.last_error()
            out.append(([u.cpu().numpy() for u in us], [np.asarray(h) for h in hists]))
        for o in out[1:]:
            for a, b in zip(o[0], out[0][0]):
                assert np.array_equal(a, b)
            for a, b in zip(o[1], out[0][1]):
                assert np.array_equal(a, b)
    ud, patches, rho_packed, p, _ = patch_case(mg, ctx, 64, (3.0, 10.0), (32, 16, 8, 4), 1e-10)
    assert {q["n"] for q in patches} >= {32, 64}
    res = []
    for tile in (3, 2, 1):
        opts = mg.mgfr_default_opts(tol=tol, precision=prec, flags=engine[1], unit_n=engine[2], tile=tile)
        up, hists, st = mg.mg_fr_solve_patches(ctx, ud, patches, dev(rho_packed), p, opts)
        assert st == mg.MGFR_OK, ctx.last_error()
        res.append((up.cpu().numpy(), [np.asarray(h) for h in hists]))
    for r in res[:2]:
        assert np.array_equal(r[0], res[2][0])
        for a, b in zip(r[1], res[2][1]):
            assert np.array_equal(a, b)
