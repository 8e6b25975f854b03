"""Wave code of the persistent workgroup-per-unit kernels, device-memory and LDS-resident
(CPU: compiles unit.hip for gfx950 to assembly, no GPU needed).

Each workgroup of those kernels loops: barrier, lane 0 takes the next unit from a device
counter into LDS, barrier, every lane reads it, solve, lane-0 stores of the results.  If the
lane-0 stores at the end of one unit and the lane-0 atomic at the start of the next are not
separated by a barrier, the compiler can join the two lane-0 branches across the loop's back
edge; the wave code then has the other lanes go round an inner loop (barrier, read the slot
again) before lane 0 has taken the next unit, and the workgroup repeats its last unit
forever.  The check: the atomic sits in the kernel's only outermost loop, behind a barrier
that comes after that loop's header, and is followed by a barrier before the slot is read."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_1110_1379_amd", "csrc", "unit.hip")
KERNELS = ["ku_whole64", "ku_whole_mixed", "kr_whole64ILi16E", "kr_whole_mixedILi16E", "kr_whole64ILi8E",
           "kr_whole_mixedILi8E", "kr_whole64ILi4E", "kr_whole_mixedILi4E"]


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "unit.s"
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out), SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out.read_text()


def body(asm, kernel):
    m = re.search(r"^(_Z\w*" + kernel + r"\w*):", asm, re.M)
    assert m, kernel
    start = m.end()
    return asm[start:asm.index(".Lfunc_end", start)].split("\n")


@pytest.mark.parametrize("kernel", KERNELS)
def test_unit_queue_atomic_sits_in_the_outer_loop_between_barriers(asm, kernel):
    lines = body(asm, kernel)
    headers = [i for i, l in enumerate(lines) if "This Loop Header: Depth=1" in l]
    assert len(headers) == 1, f"{kernel}: {len(headers)} outermost loops"
    h = headers[0]
    atomics = [i for i, l in enumerate(lines) if "global_atomic_add" in l]
    assert len(atomics) == 1, f"{kernel}: {len(atomics)} atomics"
    a = atomics[0]
    assert a > h, f"{kernel}: the atomic is outside the loop"
    # the label of the atomic's block names the loop it is in
    block = next(l for l in reversed(lines[h:a]) if re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):", l))
    assert "Depth=1" in block and "Header=" in block, f"{kernel}: atomic in {block!r}"
    assert any("s_barrier" in l for l in lines[h:a]), f"{kernel}: no barrier between loop header and atomic"
    after = lines[a:]
    barrier = next(i for i, l in enumerate(after) if "s_barrier" in l)
    read = next(i for i, l in enumerate(after) if re.search(r"\bds_read_b32\b", l))
    assert barrier < read, f"{kernel}: the slot is read before the barrier that follows the atomic"
