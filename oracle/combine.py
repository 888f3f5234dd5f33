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

The hierarchical route (Section 2.2.2) is written out as well:
`hierarchize` / `dehierarchize` are the per-grid basis changes H_l and
H_l^-1 between nodal values and hierarchical surpluses of the piecewise
linear basis, and `recombine_hier` forms H^-1 Qbar H: the surpluses of all
grids are weighted by their combination coefficients and summed per
hierarchical basis function (a node of the finest grid, shared by every
component grid that contains it), then mapped back to each grid.

Pinned by tests/test_oracle_combine.py: the combination interpolates at
every node of every component grid (the sparse-grid interpolation property),
reproduces functions that depend on one coordinate only, and is exact for
functions that lie in every component space. The hierarchical surpluses of
prod_i (x_i - lo_i)(hi_i - x_i) are prod_i h_i^2 at the level of the node
(closed form); on a lattice axis a linear function has only its level-0
coefficient; H^-1 H is the identity; the hierarchical route equals the
direct combine-then-project.
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


# ------------------------------------------------------------ hierarchical basis
def _padded(prob, l, u: np.ndarray) -> np.ndarray:
    """Nodal values on node indices J = 0 .. 2^l_i per axis, with the zero
    boundary (Dirichlet) or the zero node hi (lattice) filled in."""
    shp = grids.shape(prob, l)
    j0 = grids.first_index(prob)
    full = np.zeros(tuple(2 ** li + 1 for li in l))
    full[tuple(slice(j0, j0 + s) for s in shp)] = u.reshape(shp)
    return full


def _unpadded(prob, l, full: np.ndarray) -> np.ndarray:
    shp = grids.shape(prob, l)
    j0 = grids.first_index(prob)
    return full[tuple(slice(j0, j0 + s) for s in shp)].reshape(-1).copy()


def _axis_pass(full: np.ndarray, axis: int, li: int, inverse: bool) -> None:
    """1-D (de)hierarchization along one axis, in place. The node J at level
    k (J an odd multiple of 2^(li-k)) has the hierarchical parents
    J -/+ 2^(li-k); its surplus is its value minus their mean. Levels are
    processed finest first (forward) or coarsest first (inverse), so a
    parent always holds its nodal value when it is read."""
    levels = range(li, 0, -1) if not inverse else range(1, li + 1)
    for k in levels:
        st = 2 ** (li - k)
        J = np.arange(st, 2 ** li, 2 * st)
        mid = np.take(full, J, axis=axis)
        nb = 0.5 * (np.take(full, J - st, axis=axis) + np.take(full, J + st, axis=axis))
        idx = [slice(None)] * full.ndim
        idx[axis] = J
        full[tuple(idx)] = mid + nb if inverse else mid - nb


def hierarchize(prob, l, u: np.ndarray) -> np.ndarray:
    """H_l: nodal values -> hierarchical surpluses (grid point order)."""
    full = _padded(prob, l, u)
    for i, li in enumerate(l):
        _axis_pass(full, i, li, inverse=False)
    return _unpadded(prob, l, full)


def dehierarchize(prob, l, uh: np.ndarray) -> np.ndarray:
    """H_l^-1: hierarchical surpluses -> nodal values."""
    full = _padded(prob, l, uh)
    for i, li in enumerate(l):
        _axis_pass(full, i, li, inverse=True)
    return _unpadded(prob, l, full)


def node_keys(prob, l) -> np.ndarray:
    """Finest-grid node index of every unknown of Omega_l, as one integer
    (mixed radix 2^n + 1); it names the hierarchical basis function of the
    node, which every grid containing the node shares."""
    n = prob["n"]
    j0 = grids.first_index(prob)
    axes = [(np.arange(grids.axis_points(prob, li)) + j0) * 2 ** (n - li) for li in l]
    mesh = np.meshgrid(*axes, indexing="ij")
    key = np.zeros(mesh[0].size, dtype=np.int64)
    for m in mesh:
        key = key * (2 ** n + 1) + m.reshape(-1)
    return key


def recombine_hier(prob, grid_list, states):
    """Q = H^-1 Qbar H on the component states: combine the hierarchical
    surpluses with the combination coefficients, per basis function, then
    return to nodal values on every grid."""
    keys, vals = [], []
    for (l, _, coef), u in zip(grid_list, states):
        keys.append(node_keys(prob, l))
        vals.append(coef * hierarchize(prob, l, u))
    allk = np.concatenate(keys)
    _, inv = np.unique(allk, return_inverse=True)
    acc = np.bincount(inv, weights=np.concatenate(vals))
    out, pos = [], 0
    for (l, _, _), k in zip(grid_list, keys):
        out.append(dehierarchize(prob, l, acc[inv[pos:pos + k.size]]))
        pos += k.size
    return out
