"""Pins of the oracle's MGRIT: fixed point, finite termination, exact coarse
propagator."""
import math

import numpy as np
import pytest

from oracle import grids, mgrit, propagate
from workloads import make


def _setup(name, l, N, c, levels, **kw):
    p = make(name, **kw)
    p.update(nsteps=N, cf=c, mgrit_levels=levels)
    dt = (p["t1"] - p["t0"]) / N
    phis = [propagate.Propagator(p, l, dt * c ** k) for k in range(levels)]
    u0 = grids.initial_value(p, l)
    seq = propagate.march(p, l, u0, N, dt)
    return p, phis, u0, seq


@pytest.mark.parametrize("name,l,N,c,levels,relax", [
    ("heat2d", (4, 3), 64, 4, 2, "FCF"),
    ("heat2d", (6, 1), 64, 4, 3, "FCF"),
    ("heat3d", (3, 3, 2), 64, 8, 2, "F"),
    ("ou4d", (2, 2, 2, 2), 64, 4, 3, "FCF"),
    ("cme5d", (2, 1, 2, 1, 1), 32, 2, 2, "FCF"),
    ("varcoef6d", (2, 1, 1, 2, 1, 1), 64, 8, 2, "FCF"),
])
def test_mgrit_converges_to_sequential(name, l, N, c, levels, relax):
    # The unique solution of the space-time system is the forward solve.
    p, phis, u0, seq = _setup(name, l, N, c, levels)
    tol = 1e-14 * np.linalg.norm(u0)
    u, it, ok = mgrit.solve(phis, u0, N, c, tol, 200, relax)
    assert ok
    assert np.linalg.norm(u - seq) <= 1e-12 * np.linalg.norm(seq)


@pytest.mark.parametrize("levels,relax", [(2, "FCF"), (3, "FCF"), (2, "F"), (3, "F")])
def test_mgrit_finite_termination(levels, relax):
    # With F-relaxation each iteration makes at least one more C-point exact,
    # with FCF at least two: after k iterations the C-points 0..step*k equal
    # sequential stepping, and the last C-point is exact after ceil(M/step)
    # iterations (M = N / c coarse intervals).
    N, c = 48, 4
    M = N // c
    step = 2 if relax == "FCF" else 1
    p, phis, u0, seq = _setup("heat2d", (5, 2), N, c, levels)
    dt = (p["t1"] - p["t0"]) / N
    seq_all = propagate.march(p, (5, 2), u0, N, dt, keep_all=True)
    for k in (1, 2, 3):
        pts = []
        mgrit.solve(phis, u0, N, c, 0.0, k, relax, all_points=pts)
        for m in range(M + 1):
            err = np.linalg.norm(pts[c * m] - seq_all[c * m]) / np.linalg.norm(seq_all[c * m])
            if m <= step * k:
                assert err <= 1e-13, (k, m, err)
        # the first C-point beyond the guaranteed prefix is still inexact
        m = step * k + 1
        assert np.linalg.norm(pts[c * m] - seq_all[c * m]) > 1e-12 * np.linalg.norm(seq_all[c * m])
    u, _, _ = mgrit.solve(phis, u0, N, c, 0.0, math.ceil(M / step), relax)
    assert np.linalg.norm(u - seq) <= 1e-13 * np.linalg.norm(seq)


def test_mgrit_exact_coarse_propagator_one_iteration():
    # With Phi_coarse = Phi^c the coarse system is the exact Schur complement:
    # after one iteration every C-point is exact and the next residual vanishes.
    N, c = 32, 4
    p, phis, u0, seq = _setup("heat2d", (4, 4), N, c, 2)
    fine = phis[0]

    def exact_coarse(v):
        for _ in range(c):
            v = fine(v)
        return v

    hist = []
    u, it, ok = mgrit.solve([fine, exact_coarse], u0, N, c, 1e-13 * np.linalg.norm(u0), 5,
                            "F", history=hist)
    assert ok and it == 2
    assert hist[0] > 1e-6 and hist[1] <= 1e-13 * np.linalg.norm(u0)
    assert np.linalg.norm(u - seq) <= 1e-13 * np.linalg.norm(seq)
