"""Graph-captured domain solves (MGFR_GRAPH on mg_fr_solve) against eager cycles (needs an
MI355X).  The captured cycles are the eager cycles' kernels with the same arguments, each
ending in the stop test on the device, so the bar is bit identity: the same field, the same
residual history, the same cycle count and counters, on the capturing call and on replays of
the cached graph, for both precisions, below and above the size where the fused sweeps and
the streaming residual start, and when the cycle cap (an odd count) ends the solve."""
import sys

import numpy as np
import pytest

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


COUNTERS = ("cycles", "inner_cycles", "cell_updates", "finest_updates")


def solve(mg, ctx, rho, params, **kw):
    u, hist, st = mg.mg_fr_solve(ctx, rho, params, mg.mgfr_default_opts(**kw), raise_on_error=False)
    stats = mg.mgfr_get_stats(ctx)
    return u.cpu().numpy(), hist, st, {k: stats[k] for k in COUNTERS}


def same(a, b, what):
    ua, ha, sa, ca = a
    ub, hb, sb, cb = b
    assert sa == sb, what
    assert np.array_equal(ha, hb), (what, ha, hb)
    assert ca == cb, (what, ca, cb)
    assert np.array_equal(ua.view(np.uint64), ub.view(np.uint64)), (what, np.abs(ua - ub).max())


CASES = [(32, "fp64"), (128, "fp64"), (32, "mixed"), (128, "mixed")]


@pytest.mark.parametrize("N,prec", CASES)
def test_graph_solve_is_bitwise_eager(mg, ctx, N, prec):
    say(f"[graph] N={N} {prec}")
    precision = mg.MGFR_MIXED if prec == "mixed" else mg.MGFR_FP64
    tol = 1e-8 if prec == "mixed" else 1e-10
    rho = dev(inputs.lognormal(N, 2.0, -1.5, seed=N + 7))
    params = mg.Params(box_mpc_h=float(N), fr0_abs=1e-5)
    eager = solve(mg, ctx, rho, params, tol=tol, precision=precision, inner_cycles=2 if prec == "mixed" else 1)
    assert eager[2] == mg.MGFR_OK and eager[3]["cycles"] >= 3
    for rep in range(3):  # capture, then replays of the cached graph
        g = solve(mg, ctx, rho, params, tol=tol, precision=precision, inner_cycles=2 if prec == "mixed" else 1,
                  flags=mg.MGFR_GRAPH)
        same(eager, g, f"replay {rep}")
    # other model constants: a new capture, still the eager bits
    params2 = mg.Params(box_mpc_h=float(N), fr0_abs=1e-6)
    eager2 = solve(mg, ctx, rho, params2, tol=tol, precision=precision)
    same(eager2, solve(mg, ctx, rho, params2, tol=tol, precision=precision, flags=mg.MGFR_GRAPH), "new constants")


@pytest.mark.parametrize("N,prec", [(128, "fp64"), (128, "mixed"), (32, "mixed")])
def test_graph_solve_stops_at_the_cycle_cap(mg, ctx, N, prec):
    """An odd cycle cap ends the solve inside a replayed pair of cycles: the second cycle's
    kernels must leave the field alone (mixed at 128^3: the field then sits in the second
    buffer and is copied back)."""
    say(f"[graph cap] N={N} {prec}")
    precision = mg.MGFR_MIXED if prec == "mixed" else mg.MGFR_FP64
    rho = dev(inputs.lognormal(N, 2.0, -1.5, seed=N + 11))
    params = mg.Params(box_mpc_h=float(N), fr0_abs=1e-5)
    for cap in (3, 4):
        eager = solve(mg, ctx, rho, params, tol=1e-30, max_cycles=cap, precision=precision)
        assert eager[2] == mg.MGFR_ENOTCONV and eager[3]["cycles"] == cap
        same(eager, solve(mg, ctx, rho, params, tol=1e-30, max_cycles=cap, precision=precision, flags=mg.MGFR_GRAPH),
             f"cap {cap}")


def test_graph_solve_falls_back(mg, ctx):
    """Odd sweep counts and MGFR_PROFILE run eagerly (same bits)."""
    say("[graph] fallbacks")
    N = 64
    rho = dev(inputs.lognormal(N, 2.0, -1.5, seed=5))
    params = mg.Params(box_mpc_h=64.0, fr0_abs=1e-5)
    for kw in (dict(pre=2, post=1), dict(flags=mg.MGFR_PROFILE)):
        eager = solve(mg, ctx, rho, params, tol=1e-10, **kw)
        flags = kw.pop("flags", 0) | mg.MGFR_GRAPH
        same(eager, solve(mg, ctx, rho, params, tol=1e-10, flags=flags, **kw), str(kw))
