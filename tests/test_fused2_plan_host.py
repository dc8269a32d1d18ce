"""The two-step kernel's strip and segment plan (fused2_plan.hpp, the same
code the kernel and the host runtime use), checked on the CPU over every
height from 1 to 1300 rows and ten widths, for several SIMD counts, and on
tall lattices: output rows partition the lattice, every strip holds the
rows its second pull reaches, interior strips hold no wall row, each strip
is launched once, segments cover every column (tests/engine_host/plan_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_00185_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "engine_host")


def test_two_step_plan(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not found")
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", HARNESS, "-I", CSRC, os.path.join(HARNESS, "plan_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    assert "two-step plan: ok" in res.stdout
