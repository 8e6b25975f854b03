#!/usr/bin/env python3
"""Benchmark of the f(R) multigrid solve on one MI355X.

Default workload (halo512): one step = one complete solve of the 512^3 periodic domain
grid (box 512 Mpc/h, |f_R0| = 1e-6, lognormal sigma = 3 density plus 2000 NFW-like halos)
from the background field to an rms residual <= 1e-8, with the density already resident in
HBM.  Both solvers are timed, FP64 and mixed (FP32 correction V-cycles inside an FP64
defect-correction loop); the headline `value` is the mixed solver's cell-updates/s and
ms_per_step its time-to-tolerance, the FP64 solver is reported under "fp64".  Printed: ONE
JSON line, with the smoother's roofline position (HIP events around the finest-level
smoother launches of the timed solves, on the solve's stream) and the CPU oracle timed on a
bounded sample of the same workload.

Other workloads: --workload tophat256 | small32 (same line, other grid), amr (domain grid
plus refinement patches over 3 levels), batch (64 boxes of 64^3 + 16 of 128^3), poisson512
(the modified Poisson solve of the same 512^3 density), masked512 (a 512^3 refinement level
of oct-mask shape), tsc512 (TSC assignment and force interpolation of 512^3 particles).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "f(R) MG time-to-residual 1e-8 & cell-updates/s, 512^3, FP64 vs mixed"

# HBM bytes per finest-level (512^3) launch of the dominant kernels, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE runs scaled by a plain copy (profiles/halo512_traffic.md), with the SHA-256
# of the sources those kernels are compiled from (the kernel file, its device header and the
# by-value kernel types): when any of them differs the figure no longer describes the kernel
# that runs and `traffic` is reported as null.
MEASURED_TRAFFIC = {
    # per finest launch (one red-black sweep of the correction, 16 x 64 tiles), at 64 and 32
    # planes per workgroup
    "mixed": {"points": [({"planes": 64, "tile": 3}, 3.5597e9), ({"planes": 32, "tile": 3}, 3.0682e9)],
              "sources": {
                  "kernels_fp32.hip": "3e2d5fa7b74c8e9e8695fb1c7fd7f008127e8b020b552ac5893de6581d7cd948",
                  "fused_fp32.h": "b9ed53a6627e0abd80a493c36476053bfd8d2a934debc47118343d03e6ed03ca",
                  "device_fp32.h": "d5b6a8e51761f987af9084e51f4c3970ee35457c72c0a474d5c42afb25ff1921",
                  "kernel_types.h": "21ac1843e9d4b3e18646111fcbd3ff3b7e20b75086410058eb389d6397f79ef6"}},
    # per finest launch (one red-black sweep, 16 x 64 tiles, 128 planes per workgroup)
    "fp64": {"points": [({"planes": 128, "tile": 1}, 3.4275e9)], "sources": {
        "sweep_fp64.hip": "52fc69d7da60d3ca2f99db208d943e175ded4ad6bf8ace4cd379e03154f184c8",
        "device_fp64.h": "45739fd671f614d6a70c9201b41df3c5734bf39dd756f08db278f61fa5027ac7",
        "kernel_types.h": "21ac1843e9d4b3e18646111fcbd3ff3b7e20b75086410058eb389d6397f79ef6"}},
    # per sweep (one launch of the fused masked sweep, byte flags)
    "masked": {"bytes": 4.995e9, "sources": {
        "masked.hip": "6d044054bb4f6a7c5c48cc0c85298a8667acd115f241463a6694d6092d87489c",
        "masked_solver.hip": "966744ac3561f1ca7912ab5e2f3f4cb699879477b5a7f0d61b1cdd7d0d0be3ad",
        "device_fp64.h": "45739fd671f614d6a70c9201b41df3c5734bf39dd756f08db278f61fa5027ac7",
        "kernel_types.h": "21ac1843e9d4b3e18646111fcbd3ff3b7e20b75086410058eb389d6397f79ef6"}},
    # per pass of two sweeps
    "poisson": {"bytes": 3.6313e9, "sources": {
        "poisson_kernels.hip": "8ef270f9a78d0ee210179a3dab0de7499c9764aa3bab3ed9d665d4bd122c4738",
        "kernel_types.h": "21ac1843e9d4b3e18646111fcbd3ff3b7e20b75086410058eb389d6397f79ef6"}},
}


# HBM bytes per finest-level sweep launch of the batch workload (workgroup-per-unit engine,
# automatic sweep form), averaged over the launches of one solve at the (pre, post, inner)
# settings counted (FETCH_SIZE x 2 + WRITE_SIZE, copy-calibrated): mixed, the fused two-colour
# launches (the last of each outer iteration also adds u += e); FP64, the one-colour launches
BATCH_TRAFFIC = {
    "mixed": {"bytes": 0.4292e9, "settings": (2, 2, 3), "sources": {
        "batch_col.hip": "1c3ac948bf60869a2c8ef3224e9c0f6d227552121414c5f25f895ad53f76efdd",
        "batch.hip": "d4f88b9b651180a5616915b3f59d1d0ad76b9174d50ddcf080ec8f068b5792b9",
        "fused_fp32.h": "b9ed53a6627e0abd80a493c36476053bfd8d2a934debc47118343d03e6ed03ca",
        "device_fp32.h": "d5b6a8e51761f987af9084e51f4c3970ee35457c72c0a474d5c42afb25ff1921",
        "batch_dev.h": "de43e35ad4c4670dc0ee3196ac06e4ee6a59cd2320f45743b1b175dbf70de6f3"}},
    "fp64": {"bytes": 0.9508e9, "settings": (1, 1, 1), "sources": {
        "batch_col.hip": "1c3ac948bf60869a2c8ef3224e9c0f6d227552121414c5f25f895ad53f76efdd",
        "batch.hip": "d4f88b9b651180a5616915b3f59d1d0ad76b9174d50ddcf080ec8f068b5792b9",
        "batch_dev.h": "de43e35ad4c4670dc0ee3196ac06e4ee6a59cd2320f45743b1b175dbf70de6f3"}},
}


def batch_traffic(prec, settings=None):
    """Measured bytes per finest sweep launch of the batch workload, if the counters describe
    the kernels and tables built from these sources, at these (pre, post, inner) settings
    (without settings: at those counted)."""
    import hashlib
    entry = BATCH_TRAFFIC.get(prec)
    if entry is None or (settings is not None and tuple(settings) != tuple(entry["settings"])):
        return None
    csrc = os.path.join(ROOT, "paper_1110_1379_amd", "csrc")
    for name, digest in entry["sources"].items():
        with open(os.path.join(csrc, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    return entry["bytes"]


def _tile_shape(prec, tile):
    """Tile shape a finest-level sweep setting selects (0 is the automatic choice)."""
    if prec == "fp64":
        return "8x64" if tile == 2 else "16x64"
    return {2: "32x32", 3: "16x64", 4: "8x32", 5: "32x64"}.get(tile, "16x32")


def measured_traffic(prec, N, settings=None):
    """Bytes per finest launch if the counters describe the kernel built from these sources;
    a sweep counted at given planes and tile: at those of the timed settings (without
    settings, the first point counted)."""
    import hashlib
    entry = MEASURED_TRAFFIC.get(prec)
    if entry is None or N != 512:
        return None
    csrc = os.path.join(ROOT, "paper_1110_1379_amd", "csrc")
    for name, digest in entry["sources"].items():
        with open(os.path.join(csrc, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    if "points" not in entry:
        return entry["bytes"]
    if settings is None:
        return entry["points"][0][1]
    for want, nbytes in entry["points"]:
        if settings.get("planes") == want["planes"] and \
                _tile_shape(prec, settings.get("tile", 0)) == _tile_shape(prec, want["tile"]):
            return nbytes
    return None


WORKLOADS = {
    # name: (N, box Mpc/h, |f_R0|, generator, oracle sample (N, structures))
    "halo512": (512, 512.0, 1e-6, "halo_box", (128, 31)),
    "tophat256": (256, 256.0, 1e-5, "tophat_box", (128, 25)),
    "small32": (32, 64.0, 1e-5, "small_box", (32, 0)),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_density(name, N):
    from paper_1110_1379_amd import inputs
    gen = WORKLOADS[name][3]
    if gen == "small_box":
        return inputs.small_box(N, 0)
    if gen == "tophat_box":
        return inputs.tophat_box(N)
    return inputs.halo_box(N)


def host_cores():
    """CPUs this process may use (affinity, cgroup quota, OMP_NUM_THREADS) and the machine's
    count."""
    import oracle
    return oracle.cpu_share(), os.cpu_count()


def oracle_sample(name):
    """The bounded sample the CPU oracle runs: the same density recipe and cell size on a
    smaller periodic box (structures scaled with the volume)."""
    from paper_1110_1379_amd import inputs
    N, box, fr0, gen, (Ns, count) = WORKLOADS[name]
    box_s = box * Ns / N
    if gen == "halo_box":
        rho = inputs.halo_box(Ns, 2, count=count)
    elif gen == "tophat_box":
        rho = inputs.tophat_box(Ns, 1, count=count)
    else:
        rho = inputs.small_box(Ns, 0)
    return Ns, box_s, fr0, count, rho


def cpu_baseline(name, tol):
    """The oracle as it stands on the bounded sample, once on one host thread and once on
    every core this process may use (OpenMP); cell updates per second of each."""
    import oracle
    Ns, box_s, fr0, count, rho = oracle_sample(name)
    model = oracle.Model(box_mpc_h=box_s, fr0_abs=fr0)
    avail, total = host_cores()
    legs = {}
    for threads in (avail, 1):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        u, hist, st = oracle.solve(rho, model, oracle.Opts(tol=tol))
        dt = time.perf_counter() - t0
        legs[threads] = (oracle.last_cell_updates() / dt, dt, len(hist) - 1, st)
    oracle.set_threads(avail)
    used = oracle.threads()
    v, dt, cyc, st = legs[avail]
    v1, dt1, _, _ = legs[1]
    return {"value": v, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
            "nproc": avail, "host_cpus": total,
            "sample": f"{Ns}^3 box of {box_s:g} Mpc/h (same cell size and density recipe, "
                      f"{count} structures), FP64, solved to rms {tol:g}: {cyc} V-cycles, "
                      f"{dt:.2f} s on {used} threads (OpenMP), status {st}",
            "time_to_tol_s": dt,
            "single_thread": {"value": v1, "unit": "cell-updates/s", "cores": 1, "time_to_tol_s": dt1}}


def field_error_vs_oracle(mgfr, ctx, name, used, tol):
    """Max and rms |u - u*| of the GPU solutions (FP64 and mixed, at the timed settings and
    tolerance) against the FP64 oracle solved to rms 1e-12, on the bounded sample the CPU
    baseline runs (the oracle at the full size would take minutes)."""
    import numpy as np
    import oracle
    import torch
    Ns, box_s, fr0, count, rho = oracle_sample(name)
    ref, hist, st = oracle.solve(rho, oracle.Model(box_mpc_h=box_s, fr0_abs=fr0), oracle.Opts(tol=1e-12))
    if st != 0:
        raise SystemExit(f"oracle reference solve failed: status {st}")
    rho_d = torch.from_numpy(rho).to("cuda:0")
    params = mgfr.Params(box_mpc_h=box_s, fr0_abs=fr0)
    scale = float(np.abs(ref).max())
    out = {"sample": f"{Ns}^3 box of {box_s:g} Mpc/h (the CPU-baseline sample); oracle at rms 1e-12 "
                     f"({len(hist) - 1} V-cycles); GPU at the timed settings and tolerance {tol:g}"}
    # the oracle stopped where the timed solves stop: the same tolerance and sweep counts
    first = next(iter(used.values()))
    same, hs, st = oracle.solve(rho, oracle.Model(box_mpc_h=box_s, fr0_abs=fr0),
                                oracle.Opts(tol=tol, pre=first.pre, post=first.post))
    if st != 0:
        raise SystemExit(f"oracle same-tolerance solve failed: status {st}")
    out["same_tolerance"] = {"oracle": f"rms {tol:g}, {first.pre}+{first.post} sweeps ({len(hs) - 1} V-cycles, "
                                       f"final {hs[-1]:.3e})"}
    import ctypes
    for pname, opts in used.items():
        o = mgfr.mgfr_opts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(opts), ctypes.sizeof(o))
        o.flags = 0
        if o.planes > Ns:
            o.planes = 0
        u, h, st = mgfr.mg_fr_solve(ctx, rho_d, params, o)
        if st != mgfr.MGFR_OK:
            raise SystemExit(f"sample solve failed: {ctx.last_error()}")
        un = u.cpu().numpy()
        d = np.abs(un - ref)
        out[pname] = {"max_abs": float(d.max()), "rms_abs": float(np.sqrt(np.mean(d * d))),
                      "max_rel": float(d.max() / scale), "cycles": len(h) - 1, "final_residual": float(h[-1])}
        d2 = np.abs(un - same)
        out["same_tolerance"][pname] = {"max_abs": float(d2.max()), "rms_abs": float(np.sqrt(np.mean(d2 * d2))),
                                        "max_rel": float(d2.max() / scale)}
    return out


def time_domain(mgfr, ctx, rho_d, params, prec, tol, steps, warmup, profile=True, autotune=True,
                tune_cache=None):
    import torch
    u_d = torch.empty_like(rho_d)
    flags = mgfr.MGFR_PROFILE if profile else 0
    opts = mgfr.mgfr_default_opts(tol=tol, precision=prec, max_cycles=100, flags=flags)
    tuned = None
    if autotune:
        # untimed: the library's autotuner times sweep counts, inner cycles and planes per
        # workgroup on this very problem and the fastest setting is used below
        best, tms = mgfr.mgfr_autotune(ctx, rho_d, params, base=opts, u_scratch=u_d, cache_path=tune_cache)
        for k in mgfr.TUNED_FIELDS:
            setattr(opts, k, getattr(best, k))
        tuned = {k: getattr(best, k) for k in mgfr.TUNED_FIELDS}
        tuned["autotune_best_ms"] = tms
        log(f"autotuned prec={prec}: {tuned}")
    stream = torch.cuda.current_stream()
    for w in range(warmup):
        _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, opts, u=u_d, stream=stream)
        log(f"warmup {w} prec={prec}: status {st}, {len(hist) - 1} cycles, final {hist[-1]:.3e}")
    stats, hists = [], []
    import gc
    gc.collect()  # held off while timing (as in _timed)
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, opts, u=u_d, stream=stream)
            if st != mgfr.MGFR_OK:
                raise SystemExit(f"solve failed: {mgfr.STATUS_NAMES.get(st, st)} {ctx.last_error()}")
            stats.append(mgfr.mgfr_get_stats(ctx))
            hists.append(hist)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
    finally:
        gc.enable()
    updates = sum(s["cell_updates"] for s in stats) / steps
    finest = sum(s["finest_updates"] for s in stats) / steps
    sweep_ms = sum(s["sweep_ms"] for s in stats)
    sweep_bytes = sum(s["sweep_bytes"] for s in stats)
    launches = sum(s["sweep_launches"] for s in stats)
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None
    res = {"ms_per_step": ms, "value": updates / (ms * 1e-3), "cycles": stats[-1]["cycles"],
           "settings": tuned or {k: getattr(opts, k) for k in mgfr.TUNED_FIELDS},
           "inner_cycles": stats[-1]["inner_cycles"], "final_residual": float(hists[-1][-1]),
           "finest_cell_updates_per_s": finest / (ms * 1e-3),
           "smoother": {"achieved_GBs": achieved, "launches": launches,
                        "avg_launch_ms": sweep_ms / launches if launches else None,
                        "bytes_per_cell_sweep": 24 if prec == mgfr.MGFR_FP64 else 12}}
    log(f"prec={prec}: {ms:.2f} ms/solve, {res['cycles']} cycles, smoother "
        f"{achieved and round(achieved)} GB/s over {launches} launches")
    return res, u_d, opts


def _k32_name(settings):
    """The single-precision fused sweep the tile setting selects."""
    return {0: "k32_fused2<16, 32>", 1: "k32_fused2<16, 32>", 2: "k32_fused2<32, 32>", 3: "k32_fused2<16, 64>",
            4: "k32_fused<8, 32, 256>", 5: "k32_fused2<32, 64>"}.get(settings.get("tile", 0), "k32_fused2")


def graph_ab(mgfr, ctx, rho_d, params, opts, steps):
    """The timed configuration without event timing, with eager cycles (a host read of the
    residual after every cycle) and with MGFR_GRAPH (two cycles per captured graph, the stop
    test on the device, one flag read per replay): time per solve of each, and whether the
    two fields are the same bits.  Outside the timed region of the main metric."""
    import ctypes
    import torch
    out = {}
    fields = {}
    for name, flag in (("eager", 0), ("graph", mgfr.MGFR_GRAPH)):
        o = mgfr.mgfr_opts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(opts), ctypes.sizeof(o))
        o.flags = (o.flags & ~(mgfr.MGFR_PROFILE | mgfr.MGFR_GRAPH)) | flag
        u_d = torch.empty_like(rho_d)
        stream = torch.cuda.current_stream()

        def solve():
            _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, o, u=u_d, stream=stream)
            if st != mgfr.MGFR_OK:
                raise SystemExit(f"{name} solve failed: {mgfr.STATUS_NAMES.get(st, st)} {ctx.last_error()}")
            return hist

        ms, hist = _timed(solve, steps, 1)
        out[f"{name}_ms"] = ms
        out[f"{name}_cycles"] = len(hist) - 1
        fields[name] = u_d
    out["bitwise_equal"] = bool(torch.equal(fields["eager"], fields["graph"]))
    out["faster"] = "graph" if out["graph_ms"] < out["eager_ms"] else "eager"
    log(f"graph A/B: eager {out['eager_ms']:.2f} ms, graph {out['graph_ms']:.2f} ms, "
        f"same bits {out['bitwise_equal']}")
    return out


def stop_rule_comparison(mgfr, ctx, rho_d, params, opts, u_ref, steps=3):
    """The solve of the timed configuration stopped by the truncation-error rule of Sec. V.B
    with MLAPM's constants, rms(d) <= max(1e-6, 0.03 rms(tau)), against the field of the timed
    solve (absolute tolerance): cycles, time and the difference in u and in f_R = -e^u.  Also
    the cost of one standalone tau estimate.  Outside the timed region of the main metric."""
    import ctypes
    import torch
    o = mgfr.mgfr_opts()
    ctypes.memmove(ctypes.byref(o), ctypes.byref(opts), ctypes.sizeof(o))
    o.tol, o.tau_alpha, o.flags = 1e-6, 0.03, 0
    u_d = torch.empty_like(rho_d)
    stream = torch.cuda.current_stream()

    def solve():
        _, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, o, u=u_d, stream=stream)
        if st != mgfr.MGFR_OK:
            raise SystemExit(f"tau-rule solve failed: {mgfr.STATUS_NAMES.get(st, st)} {ctx.last_error()}")
        return hist

    ms, hist = _timed(solve, steps, 1)
    stats = mgfr.mgfr_get_stats(ctx)
    du = (u_d - u_ref).abs().max().item()
    tau_ms, (_, trms) = _timed(lambda: mgfr.mgfr_tau(ctx, rho_d, u_ref, params, stream=stream), steps, 1)
    out = {"rule": "rms(d) <= max(1e-6, 0.03 rms(tau))", "ms_per_solve": ms, "cycles": len(hist) - 1,
           "final_residual": float(hist[-1]), "tau_rms_at_stop": stats["tau_rms"],
           "max_abs_du_vs_timed_solve": du, "max_rel_dfR_vs_timed_solve": math.expm1(du),
           "tau_rms_of_timed_solution": trms, "tau_estimate_ms": tau_ms}
    log(f"tau rule: {ms:.2f} ms, {out['cycles']} cycles, max |du| {du:.3e}, tau estimate {tau_ms:.3f} ms")
    del u_d
    return out


def bench_domain(args):
    import torch
    from paper_1110_1379_amd import mgfr
    N, box, fr0, _, _ = WORKLOADS[args.workload]
    log(f"generating {args.workload} density ({N}^3)")
    rho_d = torch.from_numpy(make_density(args.workload, N)).to("cuda:0")
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    ctx = mgfr.Context(0)
    runs, fields, used = {}, {}, {}
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for p in precs:
        code = mgfr.MGFR_MIXED if p == "mixed" else mgfr.MGFR_FP64
        runs[p], fields[p], used[p] = time_domain(mgfr, ctx, rho_d, params, code, args.tol, args.steps, args.warmup,
                                         autotune=not args.no_autotune, tune_cache=args.tune_cache)
    head = runs["mixed"] if "mixed" in runs else runs["fp64"]
    headp = "mixed" if "mixed" in runs else "fp64"
    sm = head["smoother"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if headp == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N}^3 periodic, box {box:g} Mpc/h, |f_R0|={fr0:g}, n=1, "
                               f"Om=0.24, a=1; solve from the background to rms residual {args.tol:g}",
                   "N": N, "tol": args.tol, "precision": headp,
                   "pre_post": [head["settings"]["pre"], head["settings"]["post"]], "coarsest": 4,
                   "autotuned": not args.no_autotune},
        "time_to_tol_ms": head["ms_per_step"],
        "cycles": head["cycles"],
        "final_residual": head["final_residual"],
        "roofline": {
            "bound": "hbm", "achieved": sm["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (sm["achieved_GBs"] / HBM_PEAK_GBS) if sm["achieved_GBs"] else None,
            "traffic": measured_traffic(headp, N, head["settings"]),
            "kernel": (f"single-precision correction smoother {_k32_name(head['settings'])}" if headp == "mixed"
                       else "double-precision smoother k_ngs_fused") + " (finest level)",
            "bytes_per_cell": sm["bytes_per_cell_sweep"], "launches": sm["launches"],
            "avg_launch_ms": sm["avg_launch_ms"],
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
    }
    if headp == "mixed" and sm["achieved_GBs"]:
        # the correction sweep also reads its fixed base ub: 16 B per cell moved in all
        out["roofline"]["bytes_note"] = ("12 B per cell: e read and written, its right-hand side read (half the "
                                         "24 B of a double-precision sweep); the fixed base ub the correction "
                                         "sweep also reads is not credited")
        out["roofline"]["achieved_with_base"] = sm["achieved_GBs"] * 16.0 / 12.0
        out["roofline"]["frac_with_base"] = sm["achieved_GBs"] * 16.0 / 12.0 / HBM_PEAK_GBS
    for p, r in runs.items():
        r["smoother"]["traffic"] = measured_traffic(p, N, r["settings"])
        out[p] = r
    if "fp64" in runs and "mixed" in runs:
        out["speedup_mixed_over_fp64"] = runs["fp64"]["ms_per_step"] / runs["mixed"]["ms_per_step"]
        # both solves stop at the same residual; their fields differ by the error the mixed
        # solver adds (measured here, outside the timed region)
        d = (fields["mixed"] - fields["fp64"]).abs()
        ref = fields["fp64"].abs().max().item()
        out["field_error_mixed_vs_fp64"] = {
            "max_abs": d.max().item(), "rms_abs": d.square().mean().sqrt().item(),
            "max_rel": d.max().item() / ref if ref > 0 else None}
        del d
    # graph-captured cycles against eager ones, per precision, without the event timing
    if not args.no_graph_ab:
        out["graph_ab"] = {p: graph_ab(mgfr, ctx, rho_d, params, used[p], args.steps) for p in runs}
    if not args.no_stop_rule:
        out["stop_rule_comparison"] = stop_rule_comparison(mgfr, ctx, rho_d, params, used[headp], fields[headp])
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.tol)
        log("field error of the GPU solutions against the oracle on the same sample")
        out["field_error_vs_oracle"] = field_error_vs_oracle(mgfr, ctx, args.workload, used, args.tol)
    return out


def bench_poisson(args):
    """Modified Poisson solve (the potential of the density and of delta R) on the 512^3 halo
    workload, with u from an untimed mixed f(R) solve of the same density; one step = one
    Poisson solve from zero to rms residual <= tol x rms(source)."""
    import torch
    from paper_1110_1379_amd import mgfr
    N, box, fr0 = 512, 512.0, 1e-6
    log("generating halo512 density")
    rho_h = make_density("halo512", N)
    rho_d = torch.from_numpy(rho_h).to("cuda:0")
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    ctx = mgfr.Context(0)
    u_d, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, mgfr.mgfr_default_opts(
        tol=1e-8, precision=mgfr.MGFR_MIXED, inner_cycles=2, max_cycles=100))
    assert st == mgfr.MGFR_OK, ctx.last_error()
    phi = torch.empty_like(rho_d)
    opts = mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100, flags=mgfr.MGFR_PROFILE)

    def solve():
        _, h, st = mgfr.mg_poisson_solve(ctx, rho_d, u_d, params, opts, phi=phi)
        if st != mgfr.MGFR_OK:
            raise SystemExit(f"Poisson solve failed: {ctx.last_error()}")
        return h, mgfr.mgfr_get_stats(ctx)
    ms, (h, s) = _timed(solve, args.steps, args.warmup)
    achieved = s["sweep_bytes"] / (s["sweep_ms"] * 1e-3) / 1e9 if s["sweep_ms"] > 0 else None
    out = {"metric": "modified Poisson solve (phi of rho and delta R(u)), 512^3: cells/s at relative residual 1e-8",
           "value": N ** 3 / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"poisson512: {N}^3 periodic, box {box:g} Mpc/h, |f_R0|={fr0:g}; u from the "
                                  f"f(R) solve; linear V-cycles 2+2 to rms residual {args.tol:g} x rms(source)"},
           "cycles": int(len(h) - 1), "cell_updates_per_s": s["cell_updates"] / (ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS if achieved else None,
                        "traffic": measured_traffic("poisson", N),
                        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                        "kernel": "linear fused red-black sweeps kp_fused2 (finest level; two sweeps per launch, "
                                  "temporally blocked)",
                        "bytes_per_cell": 24, "sweeps_per_launch": 2,
                        "bytes_note": "24 B per cell per launch: x and S read once and x written once for both sweeps",
                        "launches": s["sweep_launches"],
                        "avg_launch_ms": s["sweep_ms"] / s["sweep_launches"] if s["sweep_launches"] else None}}
    if not args.no_cpu_baseline:
        import oracle
        from oracle import poisson as P
        from paper_1110_1379_amd import inputs
        log("timing the CPU oracle on the same density (synthetic u)")
        model = oracle.Model(box_mpc_h=box, fr0_abs=fr0)
        u = oracle.constants(model, N)["ubar"] + inputs.gaussian_field(N, 1.0, -2.0, 11)
        t0 = time.perf_counter()
        P.solve(P.source(rho_h, u, model))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N ** 3 / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole {N}^3 density with a seeded synthetic scalaron: exact periodic "
                                         f"solve by FFT in numpy (float64), {dt:.1f} s"}
    return out


def _prolong_periodic(uc):
    """Cell-centred trilinear interpolation (weights 27/9/3/1 over 64, periodic) of a coarse
    field to twice the resolution; input preparation only (the fixed values of a refinement
    level come from the coarser level's solution)."""
    import torch
    f = uc
    for d in range(3):
        even = 0.75 * f + 0.25 * torch.roll(f, 1, dims=d)
        odd = 0.75 * f + 0.25 * torch.roll(f, -1, dims=d)
        f = torch.stack([even, odd], dim=d + 1).flatten(d, d + 1)
    return f.contiguous()


def bench_masked(args):
    """A 512^3 refinement level of irregular shape solved with the mask scheme: the halo
    density, the oct mask of the densest quarter of octs plus a one-oct buffer, fixed values
    interpolated from a 256^3 solve of the restricted density (untimed set-up).  One step =
    one masked solve from those values to rms residual tol over the active cells."""
    import torch
    from paper_1110_1379_amd import inputs, mgfr
    N, box, fr0 = 512, 512.0, 1e-6
    log("generating the masked 512^3 level")
    rho_h, mask_h = inputs.masked_level(N)
    act = int((mask_h > 0).sum())
    rho_d = torch.from_numpy(rho_h).to("cuda:0")
    mask_d = torch.from_numpy(mask_h).to("cuda:0", dtype=torch.float32)
    del mask_h
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    ctx = mgfr.Context(0)
    rho_c = rho_d.reshape(N // 2, 2, N // 2, 2, N // 2, 2).mean(dim=(1, 3, 5)).contiguous()
    uc, _, st = mgfr.mg_fr_solve(ctx, rho_c, params, mgfr.mgfr_default_opts(tol=1e-8, precision=mgfr.MGFR_MIXED,
                                                                              inner_cycles=2, max_cycles=100))
    assert st == mgfr.MGFR_OK, ctx.last_error()
    u0 = _prolong_periodic(uc)
    del uc, rho_c
    u_d = torch.empty_like(u0)
    opts = mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100, flags=mgfr.MGFR_PROFILE)

    def solve():
        u_d.copy_(u0)
        _, h, st = mgfr.mg_fr_solve_masked(ctx, rho_d, mask_d, u_d, params, opts)
        if st != mgfr.MGFR_OK:
            raise SystemExit(f"masked solve failed: {ctx.last_error()}")
        return h, mgfr.mgfr_get_stats(ctx)
    ms, (h, s) = _timed(solve, args.steps, args.warmup)
    achieved = s["sweep_bytes"] / (s["sweep_ms"] * 1e-3) / 1e9 if s["sweep_ms"] > 0 else None
    sweeps = s["cycles"] * (opts.pre + opts.post)
    out = {"metric": "masked refinement level (mask scheme), 512^3: active cell-updates/s at rms residual 1e-8",
           "value": s["cell_updates"] / (ms * 1e-3), "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"masked512: {N}^3 level, box {box:g} Mpc/h, |f_R0|={fr0:g}, halo density; "
                                  f"oct mask of the densest 25% of octs plus a one-oct buffer ({act / N ** 3:.3f} "
                                  f"active); fixed values from a 256^3 solve; FAS V-cycles 2+2 to rms {args.tol:g}",
                      "active_cells": act},
           "cycles": int(len(h) - 1), "final_residual": float(h[-1]),
           "time_includes": "the 1 GiB device copy that resets u before each solve",
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS if achieved else None,
                        "traffic": measured_traffic("masked", N),
                        "traffic_unit": "HBM bytes per sweep (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                        "kernel": "masked red-black sweep km_ngs_fused, both colours in one pass (finest level)",
                        "bytes_per_sweep": "1 N^3 (the mask as byte flags: it holds only +1 and -1) + 24 per "
                                           "active cell (u read and write, density)",
                        "sweeps": sweeps, "avg_sweep_ms": s["sweep_ms"] / sweeps if sweeps else None}}
    if not args.no_cpu_baseline:
        import oracle
        Ns = 128
        log(f"timing the CPU oracle on a {Ns}^3 masked level")
        rs, ms_h = inputs.masked_level(Ns, count=31)
        model = oracle.Model(box_mpc_h=box * Ns / N, fr0_abs=fr0)
        us = oracle.constants(model, Ns)["ubar"] + 0.5 * inputs.gaussian_field(Ns, 1.0, -2.0, 44)
        t0 = time.perf_counter()
        _, hs, sts = oracle.solve_masked(rs, ms_h, model, us, oracle.Opts(tol=args.tol))
        dt = time.perf_counter() - t0
        ups = oracle.last_cell_updates()
        out["cpu_baseline"] = {"value": ups / dt, "unit": "cell-updates/s", "cores": oracle.threads(),
                               "nproc": host_cores()[0], "kind": "oracle",
                               "sample": f"{Ns}^3 masked level of {box * Ns / N:g} Mpc/h (same cell size and "
                                         f"recipe, 31 halos, {(ms_h > 0).mean():.3f} active), fixed values u_bar + "
                                         f"a smooth field, to rms {args.tol:g}: {len(hs) - 1} V-cycles, {dt:.1f} s, "
                                         f"status {sts}"}
    return out


def bench_tsc(args):
    """TSC density assignment of 512^3 clustered particles on the 512^3 grid and the TSC force
    interpolation of the potential back to them (Sec. VI.C); the potential comes from an
    untimed f(R) solve (mixed) and modified Poisson solve of the deposited density.  One step =
    one assignment + one interpolation."""
    import numpy as np
    import torch
    from paper_1110_1379_amd import inputs, mgfr
    N = Ng = 512
    box, fr0 = 512.0, 1e-6
    log("generating 512^3 particles")
    pos_h = inputs.particles(Ng, seed=3)
    npart = len(pos_h)
    # held in cell order, as a particle-mesh code keeps its particles (RAMSES links them to
    # their octs); set-up, untimed
    cell = np.floor(np.mod(pos_h * N, N)).astype(np.int64) % N
    pos_h = pos_h[np.argsort((cell[:, 0] * N + cell[:, 1]) * N + cell[:, 2], kind="stable")]
    del cell
    pos = torch.from_numpy(pos_h).to("cuda:0")
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    ctx = mgfr.Context(0)
    mass = N ** 3 / npart
    rho = mgfr.mgfr_tsc_density(ctx, pos, N, mass)
    u, _, st = mgfr.mg_fr_solve(ctx, rho, params, mgfr.mgfr_default_opts(tol=1e-8, precision=mgfr.MGFR_MIXED,
                                                                            inner_cycles=2, max_cycles=100))
    assert st == mgfr.MGFR_OK, ctx.last_error()
    phi, _, st = mgfr.mg_poisson_solve(ctx, rho, u, params, mgfr.mgfr_default_opts(tol=1e-8, max_cycles=100))
    assert st == mgfr.MGFR_OK, ctx.last_error()
    del u
    acc = torch.empty_like(pos)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    dep_ms, frc_ms = [], []

    def step():
        ev[0].record(stream)
        mgfr.mgfr_tsc_density(ctx, pos, N, mass, rho=rho, stream=stream)
        ev[1].record(stream)
        mgfr.mgfr_tsc_force(ctx, phi, pos, acc=acc, stream=stream)
        ev[2].record(stream)
        return None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        dep_ms.append(ev[0].elapsed_time(ev[1]))
        frc_ms.append(ev[1].elapsed_time(ev[2]))
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    d_ms, f_ms = sum(dep_ms) / len(dep_ms), sum(frc_ms) / len(frc_ms)
    # algorithmic bytes: assignment reads the positions and clears and fills the grid;
    # interpolation reads the positions and the potential and writes the accelerations
    dep_bytes = 24.0 * npart + 16.0 * N ** 3
    frc_bytes = 48.0 * npart + 8.0 * N ** 3
    out = {"metric": "TSC density assignment + force interpolation, 512^3 particles on 512^3: particles/s",
           "value": npart / (ms * 1e-3), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"tsc512: {npart} particles (Zel'dovich-displaced lattice, 30% in compact clumps), "
                                  f"held in cell order, on the {N}^3 grid of a {box:g} Mpc/h box; potential from the "
                                  f"f(R) and modified Poisson solves of their density",
                      "particles": npart, "N": N},
           "time_includes": "the coordinate checks of both calls (one reduction and one synchronisation each)",
           "assignment_ms": d_ms, "interpolation_ms": f_ms,
           "roofline": {"bound": "hbm", "achieved": dep_bytes / (d_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": dep_bytes / (d_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "one TSC assignment call: coordinate check, keys, radix sort, gather of offsets, "
                                  "cell table, cell sums (k_tsc_density, about 2/3 of the call)",
                        "bytes": "24 per particle + 16 per cell",
                        "traffic_note": "per-kernel FETCH/WRITE bytes of the call are listed in the TSC profile "
                                        "summary; the sort's are not counted, so no total is given",
                        "interpolation": {"achieved": frc_bytes / (f_ms * 1e-3) / 1e9,
                                          "frac": frc_bytes / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                          "bytes": "48 per particle + 8 per cell"}}}
    if not args.no_cpu_baseline:
        import oracle.tsc as T
        ns = 128
        log(f"timing the CPU oracle on {ns}^3 particles")
        ps = inputs.particles(ns, seed=3)
        t0 = time.perf_counter()
        r = T.deposit(ps, ns, 1.0)
        T.force(r, ps)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(ps) / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
                               "sample": f"{ns}^3 particles of the same recipe on the {ns}^3 grid, numpy "
                                         f"assignment + interpolation (the density as potential), {dt:.1f} s"}
    return out


def _timed(fn, steps, warmup):
    """Mean milliseconds of `steps` calls after `warmup` untimed ones.  Python's cyclic garbage
    collector is run before and held off during the timed calls: a full collection of this
    process's objects takes about 40 ms, which would otherwise land in one step at random."""
    import gc
    import torch
    for _ in range(warmup):
        fn()
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / steps, out
    finally:
        gc.enable()


def _precisions(mgfr, args):
    names = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    return [(n, mgfr.MGFR_MIXED if n == "mixed" else mgfr.MGFR_FP64) for n in names]


def _engines(args):
    return {"units": ["units"], "phases": ["phases"], "both": ["units", "phases"]}[args.engine]


def _engine_name(args):
    return {"units": "workgroup per unit", "phases": "per phase", "both": "workgroup per unit"}[args.engine]


def _batched_roofline(s, prec_name, unit_n=0, phases=False):
    """Roofline object of the batched smoother from the statistics of a solve run eagerly with
    MGFR_PROFILE: HIP events around the finest-level sweeps of the units launched per phase
    (the two colour launches of kb_ngs / kb32_ngs), algorithmic bytes of the sweeps those
    units ran."""
    launches = s["sweep_launches"]
    achieved = s["sweep_bytes"] / (s["sweep_ms"] * 1e-3) / 1e9 if s["sweep_ms"] > 0 else None
    fp64 = prec_name == "fp64"
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": None,
            "kernel": ("kc_ngs<P64> / kb_ngs (red-black Newton-Gauss-Seidel, one launch per colour: column tiles "
                       "for periodic boxes, one thread per cell for patches)" if fp64 else
                       "kf32_ngs / kb32_ngs (red-black Newton-Gauss-Seidel: periodic boxes both colours in one "
                       "pass over column tiles, two launches per pair of sweeps; patches one launch per colour, "
                       "one thread per cell)") +
                      " over the finest level of every unit" + ("" if phases else f" larger than {unit_n or 16}^3"),
            "bytes_per_cell": 24 if fp64 else 12, "launches": launches,
            "avg_launch_ms": s["sweep_ms"] / launches if launches else None,
            "timing": "one more solve of the same problem after the timed steps, launched eagerly (no graph) "
                      "with HIP events around every finest-level sweep on the solve's stream"}


def _field_error(a, b):
    d = (a - b).abs()
    ref = b.abs().max().item()
    return {"max_abs": d.max().item(), "rms_abs": d.square().mean().sqrt().item(),
            "max_rel": d.max().item() / ref if ref > 0 else None}


def bench_amr(args):
    """Domain grid (256^3, FP64) plus its refinement patches, all levels; one step = the
    patch solve of every refinement level (domain solution given), FP64 and mixed."""
    import torch
    from paper_1110_1379_amd import inputs, mgfr
    N0, box, fr0 = 256, 256.0, 1e-5
    log("generating the AMR workload")
    rho0, patches, rho_packed = inputs.amr_box(N0)
    cells = int(sum(p["n"] ** 3 for p in patches))
    log(f"{len(patches)} patches, {cells} patch cells")
    ctx = mgfr.Context(0)
    params = mgfr.Params(box_mpc_h=box, fr0_abs=fr0)
    rho_d = torch.from_numpy(rho0).to("cuda:0")
    ud, hist, st = mgfr.mg_fr_solve(ctx, rho_d, params, mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100))
    assert st == mgfr.MGFR_OK, ctx.last_error()
    rp = torch.from_numpy(rho_packed).to("cuda:0")
    runs, fields, profiled, per_phase = {}, {}, {}, {}
    for engine in _engines(args):
        for name, code in _precisions(mgfr, args):
            eflags = (mgfr.MGFR_GRAPH if args.graph else 0) | (mgfr.MGFR_PER_PHASE if engine == "phases" else 0)
            opts = mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100, precision=code, flags=eflags,
                                          unit_n=args.unit_n, tile=args.batch_sweep_tile)
            up = torch.empty_like(rp)

            def solve(opts=opts, up=up):
                _, hists, st = mgfr.mg_fr_solve_patches(ctx, ud, patches, rp, params, opts, u_packed=up)
                if st != mgfr.MGFR_OK:
                    raise SystemExit(f"patch solve failed: {ctx.last_error()}")
                return hists
            ms, hists = _timed(solve, args.steps, args.warmup)
            s = mgfr.mgfr_get_stats(ctx)
            r = {"ms_per_step": ms, "value": s["cell_updates"] / (ms * 1e-3),
                 "max_cycles_per_patch": int(max(len(h) for h in hists) - 1),
                 "max_final_residual": float(max(h[-1] for h in hists))}
            log(f"amr {engine} {name}: {ms:.2f} ms, {r['max_cycles_per_patch']} cycles max")
            if engine == "phases" and args.engine == "both":
                per_phase[name] = r
                continue

            def solve_profiled(code=code, eflags=eflags):
                pflags = mgfr.MGFR_PROFILE | (eflags & mgfr.MGFR_PER_PHASE)
                po = mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100, precision=code, flags=pflags,
                                            unit_n=args.unit_n, tile=args.batch_sweep_tile)
                _, _, st = mgfr.mg_fr_solve_patches(ctx, ud, patches, rp, params, po, u_packed=torch.empty_like(rp))
                assert st == mgfr.MGFR_OK, ctx.last_error()
                return mgfr.mgfr_get_stats(ctx)
            profiled[name] = solve_profiled
            runs[name] = r
            fields[name] = up
    headp = "mixed" if "mixed" in runs else "fp64"
    head = runs[headp]
    out = {"metric": "f(R) MG patch solve time-to-residual & cell-updates/s (AMR refinements)",
           "value": head["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if headp == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": f"amr: {N0}^3 domain (lognormal sigma 3, P ~ k^-1), {len(patches)} cube patches "
                                  f"8^3-64^3 over {max(p['level'] for p in patches)} levels "
                                  f"(contrast > 50/200/1000), {cells} patch cells, tol {args.tol:g}",
                      "precision": headp, "graph": bool(args.graph), "engine": _engine_name(args),
                      "patches": len(patches), "patch_cells": cells}}
    out.update(runs)
    if per_phase:
        out["per_phase_engine"] = per_phase
    out["roofline"] = _batched_roofline(profiled[headp](), headp, args.unit_n, args.engine == "phases")
    if len(runs) == 2:
        out["speedup_mixed_over_fp64"] = runs["fp64"]["ms_per_step"] / runs["mixed"]["ms_per_step"]
        out["field_error_mixed_vs_fp64"] = _field_error(fields["mixed"], fields["fp64"])
    if not args.no_cpu_baseline:
        import oracle
        Ns = 128
        log(f"timing the CPU oracle on the patches of a {Ns}^3 domain of the same recipe")
        r0, ps, rps = inputs.amr_box(Ns)
        m = oracle.Model(box_mpc_h=box * Ns / N0, fr0_abs=fr0)
        u0, _, st0 = oracle.solve(r0, m, oracle.Opts(tol=args.tol))  # the parent solution, untimed
        rl = [rps[p["offset"]:p["offset"] + p["n"] ** 3].reshape((p["n"],) * 3) for p in ps]
        t0 = time.perf_counter()
        _, _, sts = oracle.solve_patches(u0, ps, rl, m, oracle.Opts(tol=args.tol))
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": oracle.last_patch_updates / dt, "unit": "cell-updates/s",
                               "cores": oracle.threads(), "nproc": host_cores()[0],
                               "kind": "oracle",
                               "sample": f"the {len(ps)} patches ({sum(p['n'] ** 3 for p in ps)} cells) of a {Ns}^3 "
                                         f"domain of the same recipe and cell size, FP64, one after another to rms "
                                         f"{args.tol:g}: {dt:.1f} s, statuses {sorted(set(sts))}"}
    return out


# Sweeps before / after the coarse step and single-precision cycles per outer iteration that
# the batch workload tries per precision (the first is the library's default)
BATCH_CANDIDATES = {"mixed": [(2, 2, 1), (2, 2, 2), (2, 2, 3)], "fp64": [(2, 2, 1), (1, 1, 1), (2, 1, 1)]}


def _pick_batch_settings(name, run, args):
    """The fastest of the precision's candidates (pre, post, inner): each solved once to warm
    up, then timed as the faster of two solves.  With --no-autotune the default."""
    cands = BATCH_CANDIDATES[name]
    if args.batch_settings:
        return tuple(int(x) for x in args.batch_settings.split(",")), None
    if args.no_autotune:
        return cands[0], None
    trials = {}
    for cand in cands:
        trials["pre=%d,post=%d,inner=%d" % cand] = min(_timed(lambda: run(cand), 1, 1 if k == 0 else 0)[0]
                                                      for k in range(2))
    pick = min(cands, key=lambda c: trials["pre=%d,post=%d,inner=%d" % c])
    log(f"batch {name}: candidates {trials}, picked pre/post/inner {pick}")
    return pick, trials


def bench_batch(args):
    """64 boxes of 64^3 plus 16 of 128^3 with their own |f_R0| and sigma, solved together,
    FP64 and mixed."""
    import torch
    from paper_1110_1379_amd import inputs, mgfr
    log("generating the boxes")
    boxes = inputs.batch_boxes()
    rhos = [torch.from_numpy(b[5]).to("cuda:0") for b in boxes]
    params = [mgfr.Params(box_mpc_h=b[1], fr0_abs=b[2]) for b in boxes]
    ctx = mgfr.Context(0)
    runs, fields, profiled, per_phase, picked = {}, {}, {}, {}, {}
    for engine in _engines(args):
        for name, code in _precisions(mgfr, args):
            eflags = (mgfr.MGFR_GRAPH if args.graph else 0) | (mgfr.MGFR_PER_PHASE if engine == "phases" else 0)

            def make_opts(cand, flags, code=code):
                return mgfr.mgfr_default_opts(tol=args.tol, max_cycles=100, precision=code, flags=flags,
                                              unit_n=args.unit_n, tile=args.batch_sweep_tile, pre=cand[0],
                                              post=cand[1], inner_cycles=cand[2])
            us = [torch.empty_like(r) for r in rhos]
            if name not in picked:  # chosen with the first engine, kept for the second

                def trial(cand, eflags=eflags, us=us):
                    _, _, st = mgfr.mg_fr_solve_batch(ctx, rhos, params, make_opts(cand, eflags), us=us)
                    if st != mgfr.MGFR_OK:
                        raise SystemExit(f"batch solve failed: {ctx.last_error()}")
                picked[name] = _pick_batch_settings(name, trial, args)
            cand, trials = picked[name]
            opts = make_opts(cand, eflags)

            def solve(opts=opts, us=us):
                _, hists, st = mgfr.mg_fr_solve_batch(ctx, rhos, params, opts, us=us)
                if st != mgfr.MGFR_OK:
                    raise SystemExit(f"batch solve failed: {ctx.last_error()}")
                return hists
            ms, hists = _timed(solve, args.steps, args.warmup)
            s = mgfr.mgfr_get_stats(ctx)
            r = {"ms_per_step": ms, "value": len(boxes) / (ms * 1e-3),
                 "cell_updates_per_s": s["cell_updates"] / (ms * 1e-3),
                 "max_cycles_per_box": int(max(len(h) for h in hists) - 1),
                 "max_final_residual": float(max(h[-1] for h in hists))}
            r["settings"] = {"pre": cand[0], "post": cand[1], "inner_cycles": cand[2] if code else 1,
                             "autotuned": trials is not None}
            if trials is not None:
                r["settings"]["candidates_ms"] = trials
            log(f"batch {engine} {name}: {ms:.2f} ms, {r['max_cycles_per_box']} cycles max")
            if engine == "phases" and args.engine == "both":
                per_phase[name] = r
                continue

            def solve_profiled(cand=cand, eflags=eflags):
                pflags = mgfr.MGFR_PROFILE | (eflags & mgfr.MGFR_PER_PHASE)
                po = make_opts(cand, pflags)
                _, _, st = mgfr.mg_fr_solve_batch(ctx, rhos, params, po, us=[torch.empty_like(r) for r in rhos])
                assert st == mgfr.MGFR_OK, ctx.last_error()
                return mgfr.mgfr_get_stats(ctx)
            profiled[name] = solve_profiled
            runs[name] = r
            fields[name] = torch.cat([u.reshape(-1) for u in us])
    headp = "mixed" if "mixed" in runs else "fp64"
    head = runs[headp]
    out = {"metric": "f(R) MG batch of independent boxes: boxes/s at residual 1e-8",
           "value": head["value"], "unit": "boxes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if headp == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": "batch: 64 x 64^3 (B=64) + 16 x 128^3 (B=128), |f_R0| log-uniform "
                                  f"[1e-6,1e-4], lognormal sigma U[1,3], tol {args.tol:g}",
                      "precision": headp, "graph": bool(args.graph), "engine": _engine_name(args),
                      "pre_post_inner": [runs[headp]["settings"]["pre"], runs[headp]["settings"]["post"],
                                         runs[headp]["settings"]["inner_cycles"]]}}
    out.update(runs)
    if per_phase:
        out["per_phase_engine"] = per_phase
    roof = _batched_roofline(profiled[headp](), headp, args.unit_n, args.engine == "phases")
    if args.engine != "phases" and args.batch_sweep_tile == 0 and args.unit_n == 0 and not args.graph:
        st = runs[headp]["settings"]
        t = batch_traffic(headp, (st["pre"], st["post"], st["inner_cycles"]))
        if t is not None and roof["achieved"]:
            algo = roof["achieved"] * 1e9 * roof["avg_launch_ms"] * 1e-3
            roof["traffic"] = t
            roof["traffic_over_algorithmic"] = t / algo
            roof["traffic_note"] = ("HBM bytes per finest sweep launch averaged over one solve's launches "
                                    "(rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE, copy-calibrated); algorithmic: "
                                    f"{roof['bytes_per_cell']} B per updated cell" +
                                    ("; the last fused launch of each outer iteration also reads and writes u "
                                     "(u += e)" if headp == "mixed" else "; a colour launch writes whole "
                                     "cache lines of u and reads u and rho whole"))
    out["roofline"] = roof
    if len(runs) == 2:
        out["speedup_mixed_over_fp64"] = runs["fp64"]["ms_per_step"] / runs["mixed"]["ms_per_step"]
        out["field_error_mixed_vs_fp64"] = _field_error(fields["mixed"], fields["fp64"])
    if not args.no_cpu_baseline:
        import oracle
        sample = [b for b in boxes if b[0] == 64][:4] + [b for b in boxes if b[0] == 128][:1]
        log("timing the CPU oracle on four 64^3 boxes and one 128^3 box")
        ups, tsum, per = 0, 0.0, {64: [], 128: []}
        for N, B, fr0, _, _, rho in sample:
            t0 = time.perf_counter()
            oracle.solve(rho, oracle.Model(box_mpc_h=B, fr0_abs=fr0), oracle.Opts(tol=args.tol))
            dt = time.perf_counter() - t0
            tsum += dt
            ups += oracle.last_cell_updates()
            per[N].append(dt)
        t64, t128 = sum(per[64]) / len(per[64]), sum(per[128]) / len(per[128])
        n64 = sum(1 for b in boxes if b[0] == 64)
        n128 = len(boxes) - n64
        out["cpu_baseline"] = {"value": len(boxes) / (n64 * t64 + n128 * t128), "unit": "boxes/s",
                               "cores": oracle.threads(), "nproc": host_cores()[0],
                               "kind": "oracle", "cell_updates_per_s": ups / tsum,
                               "sample": f"four 64^3 boxes ({t64:.2f} s each on average) and one 128^3 box "
                                         f"({t128:.1f} s), FP64, to rms {args.tol:g}; boxes/s of the batch's mix "
                                         f"({n64} + {n128}) from those per-box times"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="halo512", choices=sorted(WORKLOADS) + ["amr", "batch", "poisson512", "masked512", "tsc512"])
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="domain workloads and batch: time the default options instead of tuned ones")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of autotuned settings: reused when it holds this problem, else "
                         "written after tuning (so that profiled runs time the same settings)")
    ap.add_argument("--graph", action="store_true",
                    help="amr/batch: capture one cycle's launches in a HIP graph and replay it (the default "
                         "launches every cycle eagerly, which measured as fast or faster)")
    ap.add_argument("--no-graph", action="store_true", help="amr/batch: eager launches (the default)")
    ap.add_argument("--engine", default="both", choices=["units", "phases", "both"],
                    help="amr/batch: the workgroup-per-unit engine (the line's value), the per-phase engine "
                         "(baseline), or both")
    ap.add_argument("--batch-sweep", default="auto", choices=["auto", "cell", "column", "pairs"],
                    help="amr/batch: sweeps of unit levels of side >= 32: automatic (periodic boxes over column "
                         "tiles, mixed in fused two-colour pairs; patches one thread per cell), one thread per "
                         "cell of the colour everywhere (cell), column tiles one colour per launch everywhere "
                         "(column), or as automatic with patches in fused pairs too (pairs)")
    ap.add_argument("--batch-settings", default=None,
                    help="batch: pre,post,inner to time (both precisions) instead of picking among the candidates")
    ap.add_argument("--unit-n", type=int, default=0,
                    help="amr/batch: units and levels of side <= this run in one workgroup (0: the library's 16)")
    ap.add_argument("--no-graph-ab", action="store_true",
                    help="domain workloads: skip the graph-captured against eager comparison")
    ap.add_argument("--no-stop-rule", action="store_true",
                    help="domain workloads: skip the truncation-error stop-rule comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy three times (calibrates HBM counters)")
    args = ap.parse_args()
    args.batch_sweep_tile = {"auto": 0, "cell": 1, "column": 2, "pairs": 3}[args.batch_sweep]
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each": a.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs the "
              f"solver on a single MI355X).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "amr":
        out = bench_amr(args)
    elif args.workload == "batch":
        out = bench_batch(args)
    elif args.workload == "poisson512":
        out = bench_poisson(args)
    elif args.workload == "masked512":
        out = bench_masked(args)
    elif args.workload == "tsc512":
        out = bench_tsc(args)
    else:
        out = bench_domain(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
