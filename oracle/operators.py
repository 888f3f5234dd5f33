"""Discrete spatial operators L_l on a component grid (Section 2, semi-discrete
problem u_t + L_l u = f_l; Section 4.2 heat equation; Section 4.3 master
equation; Section 4.4 Fokker-Planck equation of a linear SDE).

Every operator is a (2d+1)-point stencil assembled axis by axis: for each
unknown and each axis i the function `couplings` returns its diagonal
contribution and the coefficients of the neighbours one node below and one
node above along axis i. A neighbour that is not an unknown (a Dirichlet
boundary node, or beyond the last lattice state) is dropped, i.e. it is a
zero ghost.

Operator kinds (u_t + L u = 0 in all workloads):

  heat     L = -Laplacian: (Lu)_j = sum_i (2 u_j - u_{j+e_i} - u_{j-e_i}) / h_i^2
  varcoef  L u = -div(a grad u) in conservative form with the coefficient
           evaluated at face midpoints, a(x) = 1 + amp prod_k sin(2 pi x_k):
           (Lu)_j = -sum_i [a_{j+1/2}(u_{j+e_i}-u_j) - a_{j-1/2}(u_j-u_{j-e_i})]/h_i^2
  ou       Fokker-Planck operator of dX = -theta X dt + sigma dW (diagonal
           theta): u_t = sum_i d_i(theta_i x_i u) + (sigma^2/2) d_ii u.
           Diffusion by central differences; drift in flux form with donor-cell
           (upwind) face fluxes F_{j+1/2} = max(w,0) u_j + min(w,0) u_{j+1},
           w = -theta_i x_{j+1/2}; L is minus the discrete right-hand side.
  drift    Fokker-Planck operator of the linear SDE dX = theta X dt + sigma dW
           with a full drift matrix theta (Section 4.4): u_t = -sum_i
           d_i((theta x)_i u) + (1/2) sum_i H_ii d_ii u with H = 2 sigma D
           sigma^T diagonal (as in both systems of Section 4.4). Second-order
           finite differences, as Section 4.4.1 states for these systems:
           central diffusion, and the drift in conservative flux form with
           central face fluxes F_{j+1/2} = w_{j+1/2} (u_j + u_{j+1}) / 2, the
           face velocity w = (theta x)_i taken at the face (x_i shifted by
           -/+ h_i/2, the other coordinates at the node).
  cme      master-equation generator of independent immigration-death
           species (Section 4.3, master equation with propensities k_i and
           gamma_i x_i) on the lattice embedding with node spacing h: births
           jump +h at rate k/h, deaths jump -h at rate gamma x / h, births are
           suppressed at the last node; L = -(generator).

Pinned by tests/test_oracle_operators.py: discrete sine modes are exact
eigenvectors of heat with the closed-form eigenvalues; varcoef reduces to
heat at amp = 0, is symmetric, and is second-order consistent with
-div(a grad u) for a smooth u; ou and cme have zero column sums (exactly for
cme, away from boundary-adjacent columns for ou), the M-matrix sign pattern,
and the expected consistency order; the cme chain at h = 1 reproduces
Poisson marginals (tests/test_oracle_propagate.py); drift has zero column
sums away from the boundary (the central fluxes conserve mass), is the heat
operator times H/2 for theta = 0, is second-order consistent with the
continuous operator for a full theta, and its drift part is skew in the
interior for a constant velocity (tests/test_oracle_sde.py).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import grids


def couplings(prob, l, i: int, X: np.ndarray):
    """(diag, lower, upper) contributions of axis i at the points X (npts, d)."""
    op = prob["op"]
    h = (prob["hi"][i] - prob["lo"][i]) / 2 ** l[i]
    x = X[:, i]
    npts = X.shape[0]
    if op == "heat":
        c = np.full(npts, 1.0 / h ** 2)
        return 2.0 * c, -c, -c
    if op == "varcoef":
        amp = prob["amp"]

        def a_at(shift):
            prod = np.ones(npts)
            for k in range(X.shape[1]):
                xk = X[:, k] + (shift if k == i else 0.0)
                prod = prod * np.sin(2.0 * math.pi * xk)
            return 1.0 + amp * prod

        a_up = a_at(+0.5 * h)
        a_dn = a_at(-0.5 * h)
        return (a_up + a_dn) / h ** 2, -a_dn / h ** 2, -a_up / h ** 2
    if op == "ou":
        theta = prob["theta"][i]
        D = 0.5 * prob["sigma"] ** 2
        w_up = -theta * (x + 0.5 * h)
        w_dn = -theta * (x - 0.5 * h)
        diag = (np.maximum(w_up, 0.0) - np.minimum(w_dn, 0.0)) / h + 2.0 * D / h ** 2
        upper = np.minimum(w_up, 0.0) / h - D / h ** 2
        lower = -np.maximum(w_dn, 0.0) / h - D / h ** 2
        return diag, lower, upper
    if op == "drift":
        th = np.asarray(prob["drift"], dtype=np.float64)
        H = float(prob["diffusion"][i])
        wc = X @ th[i]  # (theta x)_i at the node
        w_up = wc + th[i, i] * 0.5 * h
        w_dn = wc - th[i, i] * 0.5 * h
        # (F_{j+1/2} - F_{j-1/2}) / h with F = w (u_j + u_{j+1}) / 2
        diag = 0.5 * (w_up - w_dn) / h + H / h ** 2
        upper = 0.5 * w_up / h - 0.5 * H / h ** 2
        lower = -0.5 * w_dn / h - 0.5 * H / h ** 2
        return diag, lower, upper
    if op == "cme":
        k = prob["k"][i]
        g = prob["gamma"][i]
        top = prob["hi"][i] - h
        not_top = (x < top - 0.5 * h).astype(np.float64)
        diag = (k / h) * not_top + g * x / h
        lower = np.full(npts, -k / h)
        upper = -g * (x + h) / h
        return diag, lower, upper
    raise ValueError(f"unknown operator kind {op!r}")


def matrix(prob, l) -> sp.csr_matrix:
    """Sparse L_l in grid point order (axis d-1 fastest)."""
    shp = grids.shape(prob, l)
    d = len(l)
    npts = int(np.prod(shp))
    X = grids.coordinates(prob, l)
    idx = np.arange(npts).reshape(shp)
    rows, cols, vals = [], [], []
    diag_total = np.zeros(npts)
    for i in range(d):
        dg, lo, up = couplings(prob, l, i, X)
        diag_total += dg
        # neighbour below along axis i
        sl_here = [slice(None)] * d
        sl_nb = [slice(None)] * d
        sl_here[i] = slice(1, None)
        sl_nb[i] = slice(None, -1)
        here = idx[tuple(sl_here)].reshape(-1)
        nb = idx[tuple(sl_nb)].reshape(-1)
        rows.append(here), cols.append(nb), vals.append(lo[here])
        # neighbour above along axis i
        sl_here[i] = slice(None, -1)
        sl_nb[i] = slice(1, None)
        here = idx[tuple(sl_here)].reshape(-1)
        nb = idx[tuple(sl_nb)].reshape(-1)
        rows.append(here), cols.append(nb), vals.append(up[here])
    rows.append(np.arange(npts)), cols.append(np.arange(npts)), vals.append(diag_total)
    L = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(npts, npts))
    return L.tocsr()


def system_matrix(prob, l, dt: float) -> sp.csr_matrix:
    """A = I + dt L_l, the matrix of one backward-Euler step (Section 2,
    time propagation: Phi = (1 + dt L)^-1; the equivalent scaled form
    (L + I/dt) u_n = u_{n-1}/dt has the same solution)."""
    L = matrix(prob, l)
    return (sp.identity(L.shape[0], format="csr") + dt * L).tocsr()


def is_symmetric(prob) -> bool:
    return prob["op"] in ("heat", "varcoef")
