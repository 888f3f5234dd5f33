"""Component grids Omega_l and the initial value on them (Section 2,
semi-discrete problem; Section 2.1.2 node counts).

Dirichlet grids: mesh width h_i = (hi_i - lo_i) / 2^{l_i}; unknowns at the
interior nodes x = lo_i + J h_i, J = 1 .. 2^{l_i} - 1; the boundary nodes
J = 0 and J = 2^{l_i} carry the homogeneous Dirichlet value 0.

Lattice grids (master equation): the integer lattice lo .. hi-1 with
hi - lo = 2^n is embedded with h_i = 2^{n - l_i}; unknowns at
x = lo + J h_i, J = 0 .. 2^{l_i} - 1 (state lo is a node on every level);
J = 2^{l_i} (the point hi) is an implicit zero node used only by the
interpolant.

Point order inside a grid: row-major, axis d-1 fastest.

Pinned by: the heat closed-form tests (node positions and sampling enter the
exact discrete solution) and the interpolation tests of oracle.combine.
"""
from __future__ import annotations

import numpy as np


def is_lattice(prob) -> bool:
    return prob["op"] == "cme"


def first_index(prob) -> int:
    """Node index J of the first unknown along every axis."""
    return 0 if is_lattice(prob) else 1


def axis_points(prob, li: int) -> int:
    return 2 ** li if is_lattice(prob) else 2 ** li - 1


def spacing(prob, l):
    return np.array([(prob["hi"][i] - prob["lo"][i]) / 2 ** l[i] for i in range(len(l))])


def axis_nodes(prob, l, i) -> np.ndarray:
    """Coordinates of the unknowns along axis i."""
    h = (prob["hi"][i] - prob["lo"][i]) / 2 ** l[i]
    J = np.arange(axis_points(prob, l[i])) + first_index(prob)
    return prob["lo"][i] + J * h


def shape(prob, l):
    return tuple(axis_points(prob, li) for li in l)


def coordinates(prob, l) -> np.ndarray:
    """Array (npts, d) of node coordinates in grid point order."""
    axes = [axis_nodes(prob, l, i) for i in range(len(l))]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def initial_value(prob, l) -> np.ndarray:
    """u0 sampled at the unknowns of Omega_l: sum_r w_r prod_i f_{r,i}(x_i),
    each factor read from the finest 1-D table at J * 2^{n - l_i}; for the
    manufactured heat problem, u*(x, t0)."""
    if prob.get("manufactured") == "heat":
        from . import manufactured
        return manufactured.u_star(coordinates(prob, l), prob["t0"])
    n = prob["n"]
    w = np.asarray(prob["ic_w"], dtype=np.float64)
    f = np.asarray(prob["ic_f"], dtype=np.float64)
    d = len(l)
    u = np.zeros(shape(prob, l))
    for r in range(len(w)):
        term = np.ones(())
        for i in range(d):
            J = np.arange(axis_points(prob, l[i])) + first_index(prob)
            fac = f[r, i, J * 2 ** (n - l[i])]
            term = np.multiply.outer(term, fac)
        u += w[r] * term
    return u.reshape(-1)
