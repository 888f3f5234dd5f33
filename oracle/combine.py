"""Combination of component solutions (Section 2.1.1, combination formula;
Section 2.2.2, recombination operator and combine-then-project operator
Q = H^-1 Qbar H).

u^(c)(x) = sum_m c_m (I_m u_m)(x), where I_m is the piecewise d-linear
interpolant on Omega_m that takes the value 0 at the Dirichlet boundary
nodes (and at the implicit node hi of a lattice axis). Summation is in
float64, grid by grid in canonical order.

Combine-then-project: in the hierarchical basis, hierarchical functions of
a level not below l vanish at every node of Omega_l, so Q applied to the
component solutions gives, at each node of Omega_l, the value of u^(c)
there. `project` evaluates that definition directly: it is the combination
sum taken at the nodes of every grid.

Pinned by tests/test_oracle_combine.py: the combination interpolates at
every node of every component grid (the sparse-grid interpolation property),
reproduces functions that depend on one coordinate only, and is exact for
functions that lie in every component space.
"""
from __future__ import annotations

import numpy as np

from . import grids


def interpolate(prob, l, u: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """(I_l u)(pts) for pts of shape (M, d)."""
    d = len(l)
    shp = grids.shape(prob, l)
    j0 = grids.first_index(prob)
    # pad with the zero boundary / zero top node so that node index J maps to
    # padded index J directly
    full = np.zeros(tuple(2 ** li + 1 for li in l))
    sl = tuple(slice(j0, j0 + s) for s in shp)
    full[sl] = u.reshape(shp)
    M = pts.shape[0]
    cell = np.empty((M, d), dtype=np.int64)
    frac = np.empty((M, d))
    for i in range(d):
        h = (prob["hi"][i] - prob["lo"][i]) / 2 ** l[i]
        t = (pts[:, i] - prob["lo"][i]) / h
        c = np.clip(np.floor(t).astype(np.int64), 0, 2 ** l[i] - 1)
        cell[:, i] = c
        frac[:, i] = t - c
    val = np.zeros(M)
    for corner in range(2 ** d):
        w = np.ones(M)
        index = []
        for i in range(d):
            bit = (corner >> (d - 1 - i)) & 1
            w = w * (frac[:, i] if bit else 1.0 - frac[:, i])
            index.append(cell[:, i] + bit)
        val += w * full[tuple(index)]
    return val


def combine_at(prob, grid_list, states, pts: np.ndarray) -> np.ndarray:
    """u^(c)(pts) = sum_m c_m (I_m u_m)(pts)."""
    out = np.zeros(pts.shape[0])
    for (l, _, coef), u in zip(grid_list, states):
        out += coef * interpolate(prob, l, u, pts)
    return out


def project(prob, grid_list, states):
    """Combine, then take the values at the nodes of every component grid."""
    return [combine_at(prob, grid_list, states, grids.coordinates(prob, l))
            for (l, _, _) in grid_list]
