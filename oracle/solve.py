"""The whole method at its fixed point (Algorithm 3, CTMGRIT^loc; Algorithm 1,
time-sequential combination method).

MGRIT inside each recombination block converges to the unique solution of
the block's space-time system (Section 2.3.1, space-time system), which is
the forward solve, i.e. time-sequential backward-Euler stepping. The plain
definition computed here is therefore Algorithm 1:

  u_l <- u0 sampled on Omega_l for every component grid
  for k = 1..s:
      if k > 1: u_l <- (combine, then project onto Omega_l)   (Section 2.2.2)
      u_l <- Phi^{N/s} u_l on every grid                       (Section 2)
  return the component states and u^(c) at requested points

The combine-and-project of the sampled initial value before the first block
is the identity at component-grid nodes (the combination interpolates at
every component node; pinned in tests/test_oracle_combine.py), so it is not
evaluated.

Pinned through its parts (index set, operators, propagator, combination) and
by the heat closed-form test of the assembled result.
"""
from __future__ import annotations

import numpy as np

from . import combine, grids, index_set, manufactured, propagate


def grid_list(prob):
    return index_set.combination_grids(prob["d"], prob["n"], prob.get("L0", 1))


def component_states(prob, grids_sel=None):
    """Final component states u_{l,N} (list, canonical order).
    grids_sel restricts to a subset of grid indices (only valid for s = 1)."""
    gl = grid_list(prob)
    s = prob.get("nrecomb", 1)
    N = prob["nsteps"]
    if N % s != 0:
        raise ValueError("nsteps must be divisible by nrecomb")
    dt = propagate.step_size(prob, 0)
    sel = range(len(gl)) if grids_sel is None else list(grids_sel)
    if s > 1 and grids_sel is not None:
        raise ValueError("grid subsets need s = 1")
    states = {g: grids.initial_value(prob, gl[g][0]) for g in sel}
    phis = {g: propagate.Propagator(prob, gl[g][0], dt) for g in sel}
    forced = manufactured.is_manufactured(prob)
    for k in range(1, s + 1):
        if k > 1:
            proj = combine.project(prob, gl, [states[g] for g in range(len(gl))])
            states = {g: proj[g] for g in sel}
        for g in sel:
            u = states[g]
            X = grids.coordinates(prob, gl[g][0]) if forced else None
            for i in range(N // s):
                if forced:
                    # u_n = Phi (u_{n-1} + dt f(t_n)), t_n = t0 + n dt
                    tn = prob["t0"] + ((k - 1) * (N // s) + i + 1) * dt
                    u = phis[g](u + dt * manufactured.forcing(X, tn))
                else:
                    u = phis[g](u)
            states[g] = u
    return [states[g] for g in sel]


def packed(states) -> np.ndarray:
    return np.concatenate([np.asarray(u).reshape(-1) for u in states])


def offsets(prob):
    gl = grid_list(prob)
    lat = grids.is_lattice(prob)
    sizes = [index_set.interior_points(l, lat) for (l, _, _) in gl]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
