"""Host-side parts of the benchmark (no GPU): the multi-GPU refusal, the
parallel oracle baseline against the single-process oracle, the traffic
record's source check and the algorithmic flop counts."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from workloads import make, targets  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_parallel_oracle_equals_single_process_oracle():
    p = make("heat2d")
    pts = targets(p, 2000, seed=0)
    t1, u1, v1 = bench.cpu_oracle(p, pts)
    t2, workers, u2, v2 = bench.cpu_oracle_parallel(p, pts, 3)
    assert workers == 3
    np.testing.assert_array_equal(u1, u2)   # same grids, same arithmetic
    np.testing.assert_allclose(v2, v1, rtol=0, atol=1e-15 * np.abs(v1).max())


def test_traffic_record_matches_its_sources():
    with open(os.path.join(ROOT, "profiles", "chain_kernel_traffic.json")) as f:
        rec = json.load(f)
    for cls, c in rec["classes"].items():
        assert bench.measured_traffic(cls) == c["bytes_per_launch"]
    assert bench.measured_traffic("W99K4") is None


def test_flops_per_iteration():
    # CG: one (2d+1)-point apply (2 flops per point), 2 dots, 3 axpys
    assert bench.flops_per_iteration(3, "cg") == 2 * 7 + 10
    # BiCGStab: two applies, 4 dots, 6 axpys
    assert bench.flops_per_iteration(2, "bicgstab") == 2 * 2 * 5 + 20
