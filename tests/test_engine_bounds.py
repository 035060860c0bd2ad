"""CPU proof of the transform engine's index rules for every supported
length and element type (persistent prefetch, early epilogue loads, LDS
addressing, launch limits, persistent work split).  A first persistent
column pass once read past its tile on the GPU in schedules whose first
radix is not the smallest; this enumeration guards every later schedule
change on the host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_engine_index_rules(tmp_path):
    exe = str(tmp_path / "engine_bounds_test")
    cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1",
           "-I", os.path.join(ROOT, "paper_2310_08408_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "engine_bounds_test.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "hold" in r.stdout
