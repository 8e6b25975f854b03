"""Builds libmgfr.so (the HIP library, gfx950) in-tree with hipcc: every source compiled to
an object in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmgfr.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["kernels_fp64.hip", "sweep_fp64.hip", "resid_fp64.hip", "prolong.hip", "kernels_fp32.hip", "batch_fp64.hip",
           "batch_fp32.hip", "batch_col.hip", "poisson_kernels.hip", "solver.hip", "batch.hip", "poisson.hip", "masked.hip",
           "masked_solver.hip", "tsc.hip", "unit.hip"]
ARCH = os.environ.get("MGFR_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        logs = list(ex.map(lambda so: _run([hipcc, *FLAGS, "-c", os.path.join(CSRC, so[0]), "-o", so[1]]),
                           zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    logs.append(_run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]))
    if verbose:
        print("".join(logs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
