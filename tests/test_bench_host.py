"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
bytes of a BRJ sweep launch and the counter record's source check."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_sweep_bytes_at_the_benchmark_workload():
    """16^3 elements, P = 3: 320 x 320 blocks; 7 sweeps, the first without the
    off-diagonal product (its iterate and face Jacobians are not read)."""
    cfg = W.config(2)
    E, nb = 4096, 320
    n = E * nb
    ctx = types.SimpleNamespace(n_elem=E, shape=(E, 5, 64), n_unknowns=n)
    faces = E * 6 * 25 * 25
    for prec, sd, sj in (("f64", 8, 8), ("f32", 4, 4), ("bf16", 2, 4)):
        blocks = E * nb * nb * sd
        per_apply = 7 * (blocks + 2 * 8 * n) + 6 * (8 * n + faces * sj)
        assert bench.sweep_bytes(ctx, cfg, prec) == pytest.approx(per_apply / 7, rel=1e-15)
    # the FP64 figure quoted with the counters: 3.4907e9 bytes per launch
    assert bench.sweep_bytes(ctx, cfg, "f64") == pytest.approx(3.4907e9, rel=1e-4)


def test_traffic_record_matches_the_sweep_source():
    """The committed counter record belongs to the current sweep source; a
    changed source voids it."""
    t = bench.measured_traffic("f64")
    assert t is not None and 3.4e9 < t < 3.6e9
    # the cylinder workload's record: 16,384 blocks of 625 x 625 doubles per launch
    t4 = bench.measured_traffic("f64", "cylinder-annulus-64x32x8-p4")
    assert t4 is not None and 5.2e10 < t4 < 6.0e10
    src = os.path.join(ROOT, "paper_2002_04222_amd", "csrc", "dgj_precond.h")
    text = open(src).read()
    orig = bench.open if hasattr(bench, "open") else None

    def fake_open(path, *a, **k):
        if os.path.abspath(path) == os.path.abspath(src):
            import io
            return io.StringIO(text + "\n// changed\n")
        return open(path, *a, **k)

    bench.open = fake_open
    try:
        assert bench.measured_traffic("f64") is None
        assert bench.measured_traffic("f64", "cylinder-annulus-64x32x8-p4") is None
    finally:
        if orig is None:
            del bench.open
        else:
            bench.open = orig


def test_residual_counter_records_match_the_kernel_sources():
    """The committed residual counter records of both workloads belong to the
    current residual sources (fused kernel, physics, shared helpers); a
    changed source voids them."""
    for name, lo, hi in (("tgv3d-16c-p3", 2.0e7, 1.0e8), ("cylinder-annulus-64x32x8-p4", 2.8e9, 4.0e9)):
        rec = bench.residual_counters(name)
        assert rec is not None, name
        assert lo < rec["traffic_bytes"] < hi and rec["fp64_flops"] > 0
    src = os.path.join(ROOT, bench.RESIDUAL_SOURCES[0])
    text = open(src).read()

    def fake_open(path, *a, **k):
        if os.path.abspath(path) == os.path.abspath(src):
            import io
            return io.StringIO(text + "\n// changed\n")
        return open(path, *a, **k)

    bench.open = fake_open
    try:
        assert bench.residual_counters("tgv3d-16c-p3") is None
    finally:
        del bench.open
