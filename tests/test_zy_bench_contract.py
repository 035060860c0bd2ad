"""The benchmark's command-line contract: one JSON line with the agreed
fields (GPU, a short run in a child process), and the one-GPU guard (CPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


@pytest.mark.gpu
def test_bench_prints_one_json_line_with_the_contract_fields():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3", "--warmup", "1",
                        "--fp64-steps", "1", "--no-cpu"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["unit"] == "grads/s"
    assert d["value"] > 0 and d["higher_is_better"] is True and d["dtype"] == "f32" and d["data"] == "synthetic"
    assert "workload" in d["config"] and d["cpu_baseline"] is None and d["errors_vs_oracle"] is None
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12 and r["launches"] == 2 * 3
    assert max(d["errors_vs_fp64"].values()) < 1e-5
    assert 0 < r["valu_frac"] < 1 and r["valu"]["unit"] == "TFLOP/s"
    sw = d["batch_sweep"]
    assert set(sw) == {"1", "32"} and all(v["value"] > 0 and v["unit"] == "grads/s" for v in sw.values())
    u = d["uneven96"]
    assert u["ms_per_replay_pair"] > 0 and 0 < u["hbm_frac"] < 1 and u["graph_launches_per_step"] == 1
