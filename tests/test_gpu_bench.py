"""The benchmark's output contract on a small workload: one JSON line with
the metric, the whole-job value, the timing fields and the roofline object of
the dominant kernel."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_contract():
    print("[case] bench.py --workload 1 --steps 2", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "1", "--steps", "2",
                        "--warmup", "1", "--no-forms", "--no-cpu-baseline", "--no-learned",
                        "--kernel-reps", "10"],
                       capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.strip().splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "tgv2d-8x8-p2"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert 0.0 < rf["frac"] <= 1.0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    # counters are recorded for the benchmark workloads only
    assert rf["traffic"] is None
    rr = d["residual_roofline"]
    assert rr["bound"] == "alu" and rr["unit"] == "TFLOP/s" and rr["peak"] == 78.6
    assert 0.0 < rr["frac"] <= 1.0 and rr["algorithmic_flops"] > 0 and rr["compulsory_bytes"] > 0
    assert d["value"] == pytest.approx(d["residual_kernel"]["dofs_per_s"])
