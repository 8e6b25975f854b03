#!/usr/bin/env python3
"""Benchmark of the f(R) multigrid solve on one MI355X.

One step = one complete solve of the 512^3 periodic domain grid (box 512 Mpc/h, |f_R0| =
1e-6, lognormal sigma = 3 density plus 2000 NFW-like halos) from the background field to an
rms residual <= 1e-8, with the density already resident in HBM.  Printed: ONE JSON line
with time-to-tolerance (ms_per_step), cell-updates/s over all multigrid levels (value), the
smoother's roofline position (HIP-event timing of the finest-level smoother launches in the
timed steps), and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed] [--workload halo512]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (N, box Mpc/h, |f_R0|, generator, oracle sample (N, count))
    "halo512": (512, 512.0, 1e-6, "halo_box", (128, 31)),
    "tophat256": (256, 256.0, 1e-5, "tophat_box", (128, 25)),
    "small32": (32, 64.0, 1e-5, "small_box", (32, 0)),
}


def make_density(name, N):
    from paper_1110_1379_amd import inputs
    gen = WORKLOADS[name][3]
    if gen == "small_box":
        return inputs.small_box(N, 0)
    if gen == "tophat_box":
        return inputs.tophat_box(N)
    return inputs.halo_box(N)


def cpu_baseline(name, tol):
    """The oracle as it stands (single thread) on a bounded sample: the same density recipe
    and cell size on a smaller periodic box (structures scaled with the volume)."""
    import oracle
    from paper_1110_1379_amd import inputs
    N, box, fr0, gen, (Ns, count) = WORKLOADS[name]
    box_s = box * Ns / N
    if gen == "halo_box":
        rho = inputs.halo_box(Ns, 2, count=count)
    elif gen == "tophat_box":
        rho = inputs.tophat_box(Ns, 1, count=count)
    else:
        rho = inputs.small_box(Ns, 0)
    t0 = time.perf_counter()
    u, hist, st = oracle.solve(rho, oracle.Model(box_mpc_h=box_s, fr0_abs=fr0), oracle.Opts(tol=tol))
    dt = time.perf_counter() - t0
    ups = oracle.last_cell_updates()
    return {"value": ups / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{Ns}^3 box of {box_s:g} Mpc/h (same cell size and density recipe, "
                      f"{count} structures), solved to rms {tol:g}: {len(hist) - 1} V-cycles, "
                      f"{dt:.1f} s, status {st}",
            "time_to_tol_s": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="halo512", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs the "
              f"solver on a single MI355X).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1110_1379_amd import mgfr

    N, box, fr0, _, _ = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload} density ({N}^3)", file=sys.stderr, flush=True)
    rho = make_density(args.workload, N)
    rho_d = torch.from_numpy(rho).to("cuda:0")
    del rho
    u_d = torch.empty_like(rho_d)
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    prec = mgfr.MGFR_MIXED if args.precision == "mixed" else mgfr.MGFR_FP64
    opts = mgfr.mgfr_default_opts(tol=args.tol, precision=prec, max_cycles=100, flags=mgfr.MGFR_PROFILE)
    ctx = mgfr.Context(0)
    stream = torch.cuda.current_stream()

    for w in range(args.warmup):
        _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, opts, u=u_d, stream=stream)
        print(f"[bench] warmup {w}: status {st}, {len(hist) - 1} cycles, final {hist[-1]:.3e}",
              file=sys.stderr, flush=True)

    stats = []
    hists = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, opts, u=u_d, stream=stream)
        if st != mgfr.MGFR_OK:
            raise SystemExit(f"solve failed: {mgfr.STATUS_NAMES.get(st, st)} {ctx.last_error()}")
        stats.append(mgfr.mgfr_get_stats(ctx))
        hists.append(hist)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    updates = sum(s["cell_updates"] for s in stats) / args.steps
    finest = sum(s["finest_updates"] for s in stats) / args.steps
    sweep_ms = sum(s["sweep_ms"] for s in stats)
    sweep_bytes = sum(s["sweep_bytes"] for s in stats)
    launches = sum(s["sweep_launches"] for s in stats)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    print(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/solve, {stats[-1]['cycles']} cycles, "
          f"smoother {achieved and round(achieved)} GB/s over {launches} launches", file=sys.stderr, flush=True)

    out = {
        "metric": "f(R) MG time-to-residual 1e-8 & cell-updates/s, 512^3, FP64 vs mixed",
        "value": updates / (ms_per_step * 1e-3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == mgfr.MGFR_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}^3 periodic, box {box:g} Mpc/h, |f_R0|={fr0:g}, n=1, "
                               f"Om=0.24, a=1; solve from the background to rms residual {args.tol:g}",
                   "N": N, "tol": args.tol, "precision": args.precision,
                   "pre_post": [opts.pre, opts.post], "coarsest": opts.coarsest_n},
        "time_to_tol_ms": ms_per_step,
        "cycles": stats[-1]["cycles"],
        "final_residual": float(hists[-1][-1]),
        "finest_cell_updates_per_s": finest / (ms_per_step * 1e-3),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
            "kernel": "finest-level Newton-Gauss-Seidel smoother",
            "launches": launches, "avg_launch_ms": sweep_ms / launches if launches else None,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.tol)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
