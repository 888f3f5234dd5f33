"""Backward-Euler propagator and time-sequential stepping (Section 2, time
propagation equation: u_{l,n} = Phi_{l,n} u_{l,n-1} + g_{l,n} with
Phi = (1 + dt L)^-1; Algorithm 1, the time-sequential combination method).

Phi is applied by a sparse direct LU factorisation of I + dt L_l (a library
primitive), factored once per grid and step size. The benchmark workloads
have f = 0, hence g_{l,n} = 0 for n >= 1; the manufactured heat problem of
Section 4.2 has g_{l,n} = Phi dt f(t_n), i.e. u_n = Phi (u_{n-1} + dt f(t_n)).

Pinned by tests/test_oracle_propagate.py: the heat closed form (discrete
sine modes are damped by exactly (1 + dt lambda)^-N), the cross-check
against the independent Krylov solvers of oracle.krylov, the exact marginal
identity for separable conservative generators, and the Poisson limit of
the lattice chain at unit spacing.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import grids, manufactured, operators


class Propagator:
    """Phi = (I + dt L_l)^-1 for one grid and one step size."""

    def __init__(self, prob, l, dt: float):
        self.A = operators.system_matrix(prob, l, dt).tocsc()
        self.lu = spla.splu(self.A)

    def __call__(self, v: np.ndarray) -> np.ndarray:
        return self.lu.solve(np.asarray(v, dtype=np.float64))


def step_size(prob, level: int = 0) -> float:
    """Time step on MGRIT level `level`: dt * c^level (Section 2.3.1,
    coarse propagator by re-discretisation with Delta T = c dt)."""
    dt = (prob["t1"] - prob["t0"]) / prob["nsteps"]
    return dt * prob["cf"] ** level


def march(prob, l, u0: np.ndarray, nsteps: int, dt: float, keep_all: bool = False,
          t_start: float | None = None):
    """u_n = Phi (u_{n-1} + dt f(t_n)), n = 1..nsteps, t_n = t_start + n dt
    (f = 0 unless the problem is the manufactured one; t_start defaults to
    t0) -- the forward solve of the space-time system, Section 2.3.1.
    Returns u_N, or all u_0..u_N."""
    phi = Propagator(prob, l, dt)
    u = np.array(u0, dtype=np.float64)
    hist = [u.copy()] if keep_all else None
    forced = manufactured.is_manufactured(prob)
    X = grids.coordinates(prob, l) if forced else None
    ts = prob["t0"] if t_start is None else t_start
    for i in range(nsteps):
        if forced:
            u = phi(u + dt * manufactured.forcing(X, ts + (i + 1) * dt))
        else:
            u = phi(u)
        if keep_all:
            hist.append(u.copy())
    return np.stack(hist) if keep_all else u


def initial_states(prob, grid_list):
    return [grids.initial_value(prob, l) for (l, _, _) in grid_list]
