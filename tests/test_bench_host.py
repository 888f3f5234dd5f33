"""Host-side parts of the benchmark (no GPU): the multi-GPU refusal, the
parallel oracle baseline against the single-process oracle, the traffic
record's source check, the one-core oracle sample, the per-grid error and the
algorithmic flop counts."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

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
    from oracle import combine, solve
    p = make("heat2d")
    pts = targets(p, 2000, seed=0)
    states = solve.component_states(p)
    u1 = solve.packed(states)
    v1 = combine.combine_at(p, solve.grid_list(p), states, pts)
    t2, workers, u2, v2 = bench.cpu_oracle_parallel(p, pts, 3)
    assert workers == 3
    np.testing.assert_array_equal(u1, u2)   # same grids, same arithmetic
    np.testing.assert_allclose(v2, v1, rtol=0, atol=1e-15 * np.abs(v1).max())


def test_one_core_sample_covers_every_layer():
    from oracle import solve
    p = make("heat3d")
    t, dof, n = bench.cpu_oracle_sample(dict(p, nsteps=4, t1=p["t1"] * 4 / p["nsteps"]),
                                        bench.SAMPLE_STRIDE)
    gl = solve.grid_list(p)
    sel = range(0, len(gl), bench.SAMPLE_STRIDE)
    assert n == len(sel) and t > 0
    assert {gl[g][2] for g in sel} == {c for (_, _, c) in gl}  # every layer's coefficient
    assert dof == sum(int(np.diff(solve.offsets(p))[g]) for g in sel)


def test_per_grid_error_sees_one_bad_grid():
    # the per-grid figure must expose a wrong small grid that the
    # whole-vector norm hides
    from oracle import solve
    p = make("heat3d")
    off = solve.offsets(p)
    ref = np.random.default_rng(0).standard_normal(off[-1])
    small = int(np.argmin(np.diff(off)))
    bad = ref.copy()
    bad[off[small]:off[small + 1]] *= 1.5
    assert bench._rel(bad, ref) < 0.05
    assert bench._per_grid_max_rel(p, bad, ref) == pytest.approx(0.5)


def test_traffic_record_follows_its_sources():
    # the committed counter record is reported while the kernel sources hash
    # to the value it was taken on, and withheld (None) once they differ
    import hashlib
    with open(os.path.join(ROOT, "profiles", "chain_kernel_traffic.json")) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    fresh = h.hexdigest() == rec["source_sha256"]
    wl = rec["workload"]
    for cls, c in rec["classes"].items():
        assert bench.measured_traffic(wl, cls) == (c["bytes_per_launch"] if fresh else None)
    assert bench.measured_traffic(wl, "W99K4/mixed") is None
    assert bench.measured_traffic("no-such-workload", next(iter(rec["classes"]))) is None


def test_flops_per_iteration():
    # CG: one (2d+1)-point apply (2 flops per point), 2 dots, 3 axpys
    assert bench.flops_per_iteration(3, "cg") == 2 * 7 + 10
    # BiCGStab: two applies, 4 dots, 6 axpys
    assert bench.flops_per_iteration(2, "bicgstab") == 2 * 2 * 5 + 20
