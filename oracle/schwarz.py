"""Two-level overlapping Schwarz preconditioner of the spatial solver
(Section 2.1.2, spatial subproblem solver by domain decomposition; solver
settings Section 4.1). Test infrastructure: a plain dense statement of the
preconditioner on small grids.

For a component grid Omega_l and the matrix A = I + dt L_l of one implicit
step:

  ordering   every unknown is placed on the isotropic lattice of the grid's
             largest level Lmax by virtual nodes (unknown J of axis i sits at
             lattice coordinate J 2^(Lmax - l_i)); the unknowns are ordered by
             the index of their lattice point along a d-dimensional Hilbert
             curve of order Lmax. The curve is Skilling's ("Programming the
             Hilbert curve", AIP Conf. Proc. 707, 2004): the coordinates are
             turned into the curve's transposed index by his axes-to-
             transpose recurrence and the index bits read off interleaved.
  partition  P = ceil(N / 2^S) disjoint subdomains of consecutive curve
             positions, N - P w of size w + 1 first and the rest of size
             w = floor(N / P).
  overlap    with gamma = m / 2 each disjoint subdomain is extended by
             floor(gamma w) positions on each side of the curve (clipped at
             its ends); for gamma = 1/2 the points within floor(w / 2) of an
             interior subdomain boundary lie in two extended subdomains (all
             points when w is even, all but one per subdomain when it is
             odd), and subdomains two apart never overlap. R_i is the
             injection onto the extended subdomain.
  weights    D_i = omega_i I, omega_i = 1 / (the largest number of extended
             subdomains holding a point of the disjoint subdomain i).
  coarse     each disjoint subdomain is cut into q consecutive blocks (sizes
             differing by at most one, larger first; q = 2^(S - 4) unless
             given, at most the subdomain size); R_0 has one row of ones per
             block; A_0 = R_0 A R_0^T, F = R_0^T A_0^-1 R_0.
  one-level  C1 = sum_i R_i^T D_i (R_i A R_i^T)^-1 R_i
  additive   C_add = C1 + F                       (with BiCGStab)
  balanced   C_bal = G^T C1 G + F, G = I - A F    (with CG)

Library primitives: numpy's dense inverse and products.

Pinned by tests/test_oracle_schwarz.py: the curve visits every lattice point
once and consecutive points are lattice neighbours (the Hilbert property,
d = 1..4); partition sizes and counts as Section 2.1.2 states; overlap
multiplicity two near interior boundaries and never above two; F A F = F; C_bal equals A^-1 exactly
for one subdomain and when the coarse space holds every point; C_bal is
symmetric positive definite for a symmetric positive definite A; the
preconditioned CG of oracle.krylov reaches the direct solution in fewer
iterations than plain CG.
"""
from __future__ import annotations

import math

import numpy as np

from . import grids, operators


def hilbert_index(coords, bits: int) -> int:
    """Index along the d-dimensional Hilbert curve of order `bits` of the
    lattice point `coords` (each in [0, 2^bits))."""
    X = [int(c) for c in coords]
    n = len(X)
    if bits <= 0 or n == 0:
        return 0
    M = 1 << (bits - 1)
    # inverse undo of the reflections and exchanges, most significant first
    Q = M
    while Q > 1:
        P = Q - 1
        for i in range(n):
            if X[i] & Q:
                X[0] ^= P
            else:
                t = (X[0] ^ X[i]) & P
                X[0] ^= t
                X[i] ^= t
        Q >>= 1
    # Gray encoding
    for i in range(1, n):
        X[i] ^= X[i - 1]
    t = 0
    Q = M
    while Q > 1:
        if X[n - 1] & Q:
            t ^= Q - 1
        Q >>= 1
    for i in range(n):
        X[i] ^= t
    # the transposed index, bits interleaved from the top
    h = 0
    for b in range(bits - 1, -1, -1):
        for i in range(n):
            h = (h << 1) | ((X[i] >> b) & 1)
    return h


def lattice_coordinates(prob, l) -> np.ndarray:
    """(npts, d) isotropic lattice coordinates of the unknowns (virtual nodes
    between them), in grid point order."""
    lmax = max(l)
    axes = []
    for i, li in enumerate(l):
        J = np.arange(grids.axis_points(prob, li)) + grids.first_index(prob)
        axes.append(J * 2 ** (lmax - li))
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def curve_order(prob, l) -> np.ndarray:
    """Grid point indices in Hilbert-curve order."""
    C = lattice_coordinates(prob, l)
    keys = [hilbert_index(c, max(l)) for c in C]
    return np.argsort(np.array(keys, dtype=np.int64), kind="stable")


class Decomposition:
    """Subdomains, weights and coarse blocks of one grid (positions along
    the curve; `order` maps positions to grid point indices)."""

    def __init__(self, prob, l, S: int, gamma: float = 0.5, q: int | None = None):
        self.order = curve_order(prob, l)
        N = len(self.order)
        self.N = N
        P = max(1, math.ceil(N / 2 ** S))
        w = N // P
        big = N - P * w
        sizes = [w + 1] * big + [w] * (P - big)
        starts = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        self.P = P
        self.disjoint = [(int(starts[i]), int(starts[i + 1])) for i in range(P)]
        ov = int(math.floor(gamma * w)) if P > 1 else 0
        self.extended = [(max(0, a - ov), min(N, b + ov)) for a, b in self.disjoint]
        mult = np.zeros(N, dtype=int)
        for a, b in self.extended:
            mult[a:b] += 1
        self.multiplicity = mult
        self.omega = [1.0 / mult[a:b].max() for a, b in self.disjoint]
        if q is None:
            q = 2 ** (S - 4) if S >= 4 else 1
        q = max(1, int(q))
        blocks = []
        for a, b in self.disjoint:
            n = b - a
            nb = min(q, n)
            bw, bbig = n // nb, n - nb * (n // nb)
            bs = [bw + 1] * bbig + [bw] * (nb - bbig)
            cur = a
            for s in bs:
                blocks.append((cur, cur + s))
                cur += s
        self.blocks = blocks

    def restriction(self, a: int, b: int) -> np.ndarray:
        """Injection R (rows: positions a..b-1) as a dense matrix."""
        R = np.zeros((b - a, self.N))
        R[np.arange(b - a), self.order[a:b]] = 1.0
        return R

    def coarse_restriction(self) -> np.ndarray:
        R0 = np.zeros((len(self.blocks), self.N))
        for k, (a, b) in enumerate(self.blocks):
            R0[k, self.order[a:b]] = 1.0
        return R0


def one_level(A: np.ndarray, dec: Decomposition) -> np.ndarray:
    """C1 = sum_i R_i^T omega_i (R_i A R_i^T)^-1 R_i (dense)."""
    C = np.zeros_like(A)
    for (a, b), om in zip(dec.extended, dec.omega):
        R = dec.restriction(a, b)
        C += om * R.T @ np.linalg.inv(R @ A @ R.T) @ R
    return C


def coarse(A: np.ndarray, dec: Decomposition) -> np.ndarray:
    """F = R_0^T (R_0 A R_0^T)^-1 R_0 (dense)."""
    R0 = dec.coarse_restriction()
    return R0.T @ np.linalg.inv(R0 @ A @ R0.T) @ R0


def additive(A: np.ndarray, dec: Decomposition) -> np.ndarray:
    return one_level(A, dec) + coarse(A, dec)


def balanced(A: np.ndarray, dec: Decomposition) -> np.ndarray:
    F = coarse(A, dec)
    G = np.eye(A.shape[0]) - A @ F
    return G.T @ one_level(A, dec) @ G + F


def preconditioner(prob, l, dt: float, S: int, form: str | None = None) -> np.ndarray:
    """The dense preconditioner of grid l for the step matrix I + dt L_l:
    balanced with CG (symmetric operators), additive with BiCGStab
    (Section 4.1), unless `form` names one."""
    A = operators.system_matrix(prob, l, dt).toarray()
    dec = Decomposition(prob, l, S)
    if form is None:
        form = "balanced" if prob.get("krylov", "cg") == "cg" else "additive"
    return balanced(A, dec) if form == "balanced" else additive(A, dec)
