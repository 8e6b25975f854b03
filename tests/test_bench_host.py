"""Host logic of bench.py that runs without a GPU: the one-GPU guard, the source-hash guard
on the measured HBM traffic, and the roofline arithmetic of the batched smoother."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def digest(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    # the committed figures describe the committed sources
    for prec, entry in bench.MEASURED_TRAFFIC.items():
        first = entry["points"][0][1] if "points" in entry else entry["bytes"]
        assert bench.measured_traffic(prec, 512) == first, prec
        assert bench.measured_traffic(prec, 256) is None
    assert bench.measured_traffic("tsc", 512) is None
    # a figure taken at given planes and tile holds only for those (tile 0 is the automatic shape)
    for prec, entry in bench.MEASURED_TRAFFIC.items():
        for want, nbytes in entry.get("points", []):
            assert bench.measured_traffic(prec, 512, dict(want)) == nbytes, prec
            assert bench.measured_traffic(prec, 512, dict(want, planes=3 * want["planes"])) is None, prec
            other = next(t for t in range(6) if bench._tile_shape(prec, t) != bench._tile_shape(prec, want["tile"]))
            assert bench.measured_traffic(prec, 512, dict(want, tile=other)) is None, prec
    assert bench._tile_shape("fp64", 0) == bench._tile_shape("fp64", 1) == "16x64"
    assert bench._tile_shape("mixed", 0) == bench._tile_shape("mixed", 1) == "16x32"
    # a changed source voids the figure of every kernel built from it, and only those
    csrc = tmp_path / "paper_1110_1379_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1110_1379_amd", "csrc"), csrc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", {
        "a": {"bytes": 1.0, "sources": {"kernels_fp64.hip": digest(csrc / "kernels_fp64.hip"),
                                        "kernel_types.h": digest(csrc / "kernel_types.h")}},
        "b": {"bytes": 2.0, "sources": {"kernels_fp32.hip": digest(csrc / "kernels_fp32.hip"),
                                        "kernel_types.h": digest(csrc / "kernel_types.h")}},
        **bench.MEASURED_TRAFFIC})
    for edited in sorted({name for e in bench.MEASURED_TRAFFIC.values() for name in e["sources"]}):
        before = {p: bench.measured_traffic(p, 512) for p in bench.MEASURED_TRAFFIC}
        with open(csrc / edited, "a") as fh:
            fh.write("\n// edited\n")
        for prec, entry in bench.MEASURED_TRAFFIC.items():
            got = bench.measured_traffic(prec, 512)
            if edited in entry["sources"]:
                assert got is None, (edited, prec)
            else:
                assert got == before[prec], (edited, prec)


def test_batch_traffic_follows_the_sources(tmp_path, monkeypatch):
    # the committed batch figures describe the committed sources; an edit to any voids them
    for prec, entry in bench.BATCH_TRAFFIC.items():
        assert bench.batch_traffic(prec) == entry["bytes"], prec
        assert bench.batch_traffic(prec, entry["settings"]) == entry["bytes"], prec
        other = tuple(entry["settings"][:2]) + (entry["settings"][2] + 1,)
        assert bench.batch_traffic(prec, other) is None, prec
    assert bench.batch_traffic("masked") is None
    csrc = tmp_path / "paper_1110_1379_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1110_1379_amd", "csrc"), csrc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for edited in sorted({name for e in bench.BATCH_TRAFFIC.values() for name in e["sources"]}):
        before = {p: bench.batch_traffic(p) for p in bench.BATCH_TRAFFIC}
        with open(csrc / edited, "a") as fh:
            fh.write("\n// edited\n")
        for prec, entry in bench.BATCH_TRAFFIC.items():
            got = bench.batch_traffic(prec)
            assert got == (None if edited in entry["sources"] else before[prec]), (edited, prec)


@pytest.mark.parametrize("prec,bpc", [("fp64", 24), ("mixed", 12)])
def test_batched_roofline(prec, bpc):
    s = {"sweep_launches": 8, "sweep_ms": 2.0, "sweep_bytes": 4.0e9}
    r = bench._batched_roofline(s, prec)
    assert r["achieved"] == pytest.approx(2000.0)  # 4 GB in 2 ms
    assert r["frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS)
    assert r["avg_launch_ms"] == pytest.approx(0.25)
    assert r["bytes_per_cell"] == bpc and r["bound"] == "hbm" and r["traffic"] is None
    empty = bench._batched_roofline({"sweep_launches": 0, "sweep_ms": 0.0, "sweep_bytes": 0.0}, prec)
    assert empty["achieved"] is None and empty["frac"] is None and empty["avg_launch_ms"] is None
