"""mg_fr_solve_noalloc, the domain solve for callers that cannot allocate (needs an MI355X):
through the C ABI it must give what mg_fr_solve gives on the same input, bit for bit (the same
kernels on the same data; only the scratch addresses differ), on two calls in a row with the
second one smaller, in double precision and mixed precision; sizes beyond its fixed array,
MGFR_PROFILE and MGFR_GRAPH are refused."""
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgfr.lib()
    return mgfr


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_solve_equals_the_allocating_solve(mg, precision):
    import torch
    prec = mg.MGFR_MIXED if precision == "mixed" else mg.MGFR_FP64
    tol = 1e-8 if precision == "mixed" else 1e-11
    ctx_a = mg.Context(0)   # mg_fr_solve: its own scratch
    ctx_b = mg.Context(0)   # mg_fr_solve_noalloc: the library's fixed array
    try:
        for N, box, fr0, seed in ((128, 128.0, 1e-5, 31), (32, 64.0, 1e-6, 32)):
            say(f"[noalloc] {precision} N={N}")
            rho = dev(inputs.tophat_box(N, seed, count=max(1, N // 8)))
            p = mg.Params(box_mpc_h=box, fr0_abs=fr0)
            o = mg.mgfr_default_opts(tol=tol, precision=prec, inner_cycles=2 if precision == "mixed" else 1)
            ua, ha, sa = mg.mg_fr_solve(ctx_a, rho, p, o)
            ub = torch.full_like(rho, float("nan"))
            ub, hb, sb = mg.mg_fr_solve_noalloc(ctx_b, rho, ub, p, o)
            assert sa == mg.MGFR_OK and sb == mg.MGFR_OK, (ctx_a.last_error(), ctx_b.last_error())
            assert np.array_equal(ha, hb), (ha, hb)
            torch.cuda.synchronize()
            assert torch.equal(ua, ub)
            st_a, st_b = mg.mgfr_get_stats(ctx_a), mg.mgfr_get_stats(ctx_b)
            for k in ("cycles", "inner_cycles", "cell_updates", "finest_updates"):
                assert st_a[k] == st_b[k], k
    finally:
        ctx_a.close()
        ctx_b.close()


def test_noalloc_refuses_what_it_cannot_hold(mg):
    import torch
    ctx = mg.Context(0)
    try:
        p = mg.Params(box_mpc_h=256.0)
        rho = torch.ones((256,) * 3, dtype=torch.float64, device="cuda:0")
        u = torch.empty_like(rho)
        _, _, st = mg.mg_fr_solve_noalloc(ctx, rho, u, p, raise_on_error=False)
        assert st == mg.MGFR_EINVAL and "128" in ctx.last_error()
        rho = torch.ones((16,) * 3, dtype=torch.float64, device="cuda:0")
        u = torch.empty_like(rho)
        for flag in (mg.MGFR_PROFILE, mg.MGFR_GRAPH):
            _, _, st = mg.mg_fr_solve_noalloc(ctx, rho, u, p, mg.mgfr_default_opts(flags=flag), raise_on_error=False)
            assert st == mg.MGFR_EINVAL, flag
        # a valid call after the refusals works
        _, h, st = mg.mg_fr_solve_noalloc(ctx, rho, u, p, mg.mgfr_default_opts(tol=1e-12), raise_on_error=False)
        assert st == mg.MGFR_OK and len(h) == 1          # uniform density: the background solves it
    finally:
        ctx.close()
