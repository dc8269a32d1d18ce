"""Host logic of bench.py (no GPU): the refusal of more than one GPU, the
algorithmic byte counts behind the roofline, the lookup of the measured HBM
traffic (keyed by the fused kernel's sources and the lattice), the average
launch duration from the two bracketing events, and the CPU oracle leg."""
import json
import os
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
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_kernel():
    lx, ly = 2048, 8192
    sites = lx * ly
    k = bench.kernel_bandwidth({name: {"avg_ms": 1.0} for name in
                                ("fused", "propagate", "collide", "bc", "pbc", "fused_bulk",
                                 "fused_border")}, sites, lx, ly)
    # one read and one write of all 37 binary64 populations per site
    assert k["fused"]["algorithmic_bytes"] == 592 * sites == 9932111872
    assert k["propagate"]["algorithmic_bytes"] == k["collide"]["algorithmic_bytes"] == 592 * sites
    assert k["bc"]["algorithmic_bytes"] == 592 * 6 * lx           # 3 + 3 wall rows
    assert k["pbc"]["algorithmic_bytes"] == 2 * 52 * ly * 8        # 26 runs per side, read + write
    assert k["fused_bulk"]["algorithmic_bytes"] + k["fused_border"]["algorithmic_bytes"] == 592 * sites
    assert k["fused"]["gbs"] == pytest.approx(9932111872 / 1e-3 / 1e9)
    assert k["fused"]["hbm_frac"] == pytest.approx(k["fused"]["gbs"] / 8000.0)
    half = bench.kernel_bandwidth({"fused": {"avg_ms": 1.0}}, sites, lx, ly, elem_bytes=4)
    assert half["fused"]["algorithmic_bytes"] == 296 * sites


def test_average_launch_from_bracketing_events():
    k = bench.single_kernel("fused", {"span_ms": 1675.0}, 1000)
    assert k["fused"]["launches"] == 1000
    assert k["fused"]["avg_ms"] == pytest.approx(1.675)


def test_measured_traffic_is_keyed_by_sources_and_lattice(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["lx"] == 2048 and rec["ly"] == 8192 and rec["layout"] == "column"
    # used only while it matches the kernel sources as they stand
    current = rec["kernel_source_sha"] == bench.kernel_source_sha()
    assert bench.measured_traffic(2048, 8192, "column") == (rec["bytes_per_launch"] if current else None)
    assert bench.measured_traffic(2048, 8192, "planar") is None
    assert bench.measured_traffic(1024, 8192, "column") is None
    # a record taken from other sources is not used
    stale = dict(rec, kernel_source_sha="0" * 16)
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic(2048, 8192, "column") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(2048, 8192, "column") is None


def test_cpu_baseline_reports_the_oracle():
    out = bench.cpu_baseline(0.0, small_steps=2)  # one step of the strip, 2 of 64 x 128
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS" and out["cores"] == 1
    assert out["value"] > 0
    assert "2048x256" in out["sample"]
    assert out["small_lattice_64x128"]["steps"] == 2 and out["small_lattice_64x128"]["mlups"] > 0
