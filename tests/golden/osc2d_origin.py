"""Writes osc2d_origin.npz: the oracle's time-sequential component states of
the two-dimensional oscillator (Section 4.4.1; L = 14, L0 = 6, dt = 0.005,
20,000 backward-Euler steps to T = 100) sampled at the spatial origin every
EVERY steps, one row per component grid, plus the combination coefficients.
Calls only the oracle and the seeded workload builder.

    python tests/golden/osc2d_origin.py            # writes the .npz beside it
"""
from __future__ import annotations

import os
import sys
from multiprocessing import get_context

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NSTEPS = 20000
DT = 0.005
EVERY = 40
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "osc2d_origin.npz")


def problem():
    from workloads import make
    p = make("fp_osc2d", n=14, L0=6, prec="fp64")
    p["t1"] = NSTEPS * DT
    p["nsteps"] = NSTEPS
    return p


def origin_series(g: int, nsteps: int = NSTEPS) -> np.ndarray:
    """u_{l,n}(0) for n = 0, EVERY, 2 EVERY, ..., nsteps on grid g."""
    from oracle import grids, propagate, solve
    p = problem()
    l = solve.grid_list(p)[g][0]
    phi = propagate.Propagator(p, l, DT)
    u = grids.initial_value(p, l)
    X = grids.coordinates(p, l)
    io = int(np.argmin(np.abs(X).sum(axis=1)))
    if np.abs(X[io]).max() != 0.0:
        raise RuntimeError("the origin is not a node of the grid")
    out = [u[io]]
    for i in range(nsteps):
        u = phi(u)
        if (i + 1) % EVERY == 0:
            out.append(u[io])
    return np.array(out)


def compute(workers: int | None = None, nsteps: int = NSTEPS):
    """(levels, coefficients, series[grid, sample]) from the oracle."""
    from oracle import solve
    gl = solve.grid_list(problem())
    with get_context("spawn").Pool(workers or len(gl)) as pool:
        series = pool.starmap(origin_series, [(g, nsteps) for g in range(len(gl))])
    return (np.array([l for (l, _, _) in gl]), np.array([c for (_, _, c) in gl], dtype=float),
            np.stack(series))


if __name__ == "__main__":
    levels, coef, series = compute()
    np.savez(OUT, levels=levels, coef=coef, series=series, every=EVERY, dt=DT)
    print(f"wrote {OUT}: {series.shape[0]} grids x {series.shape[1]} samples")
