"""CPU checks of the benchmark's host-side helpers (no GPU)."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import hmgref as O  # noqa: E402


def test_objective_helpers_match_the_oracle():
    C = np.random.default_rng(1).standard_normal((6, 6))
    assert np.array_equal(bench.bulk_weights(), O.bulk_weights())
    assert abs(bench.bulk_modulus(C) - O.bulk_modulus(C)) < 1e-14


def test_source_digest_ignores_comments_only(tmp_path):
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {  // one\n  return x + 1;\n}\n/* block\n comment */\n")
    b = tmp_path / "b.hip"
    b.write_text("// header\nint f(int x) {\n\n  return x + 1;  // changed remark\n}\n")
    c = tmp_path / "c.hip"
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.source_hash([str(a)]) == bench.source_hash([str(b)])
    assert bench.source_hash([str(a)]) != bench.source_hash([str(c)])


def test_committed_traffic_scales_with_the_launch():
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t["source_sha256_16"] != bench.source_hash():
        assert bench.measured_traffic("matvec", 1.0) is None
        pytest.skip("the traffic summary was taken on other kernel sources")
    k = t["kernels"]["matvec"]
    # scaled to a launch with half the algorithmic bytes (three active cases)
    half = bench.measured_traffic("matvec", 0.5 * k["algorithmic_bytes_per_launch"])
    assert abs(half - 0.5 * k["hbm_bytes_per_launch"]) < 1e-6 * k["hbm_bytes_per_launch"]
    assert bench.measured_traffic("no_such_kernel", 1.0) is None


def test_more_than_one_gpu_is_refused_before_any_device_use():
    import subprocess
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300,
                         env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert res.returncode == 2
    assert "one GPU" in res.stdout + res.stderr
    assert res.stdout.strip() == "" or not res.stdout.lstrip().startswith("{")
