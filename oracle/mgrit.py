"""Multigrid reduction in time (Section 2.3.1; Algorithm 2 and the remark on
linearity after it; multilevel by recursion, Section 2.3.1 overview).

The time grid t_0..t_N is split into C-points (multiples of the coarsening
factor c) and F-points. On level k the propagator is Phi_k with step
dt * c^k (re-discretisation, Section 2.3.1). One cycle on level k for the
block bidiagonal system  e_0 = g_0,  e_n - Phi_k e_{n-1} = g_n  is

  1. relaxation: F-relaxation, then (for FCF) C-relaxation and a second
     F-relaxation (Section 2.3.1, relaxation schemes);
  2. restriction by injection of the residual at the C-points,
     r_m = g_{cm} + Phi_k e_{cm-1} - e_{cm}  (r_0 = g_0 - e_0);
  3. coarse solve of the level-(k+1) system with right-hand side r: exactly
     (sequential forward solve) on the coarsest level, otherwise one cycle
     from a zero initial guess;
  4. correction e_{cm} += e^coarse_m, followed on intermediate levels by an
     F-relaxation (prolongation = injection followed by F-relaxation).

Because the operator is linear, step 3 solves directly for the coarse error
(the linear form described after Algorithm 2); its iterates equal those of
the FAS form in exact arithmetic.

On level 0 the unknowns are u_0..u_N with u_0 = u0 and f = 0; the initial
guess is u0 at every time point; iteration stops once
max_m ||r_m||_2 <= tol (Section 4.1: all spatial l2 norms below the
tolerance), checked after the relaxation of each iteration.

Pinned by tests/test_oracle_mgrit.py: the converged iterate equals
sequential stepping; finite termination after ceil(M/2) FCF iterations
(M coarse intervals) for two and three levels; one-iteration convergence
when the coarse propagator is the exact Phi^c.
"""
from __future__ import annotations

import numpy as np


def _f_relax(phi, e, g, c):
    N = len(e) - 1
    for m in range(N // c):
        for j in range(1, c):
            n = c * m + j
            e[n] = phi(e[n - 1]) + g[n]


def _c_relax(phi, e, g, c):
    N = len(e) - 1
    for m in range(1, N // c + 1):
        n = c * m
        e[n] = phi(e[n - 1]) + g[n]


def _relax(phi, e, g, c, relax):
    _f_relax(phi, e, g, c)
    if relax == "FCF":
        _c_relax(phi, e, g, c)
        _f_relax(phi, e, g, c)


def _residual(phi, e, g, c):
    N = len(e) - 1
    r = [g[0] - e[0]]
    for m in range(1, N // c + 1):
        n = c * m
        r.append(g[n] + phi(e[n - 1]) - e[n])
    return r


def _cycle(phis, k, g, c, relax):
    """One cycle on level k for e_0 = g_0, e_n = Phi_k e_{n-1} + g_n from a
    zero initial guess; returns all N_k + 1 values."""
    N = len(g) - 1
    e = [np.zeros_like(g[0]) for _ in range(N + 1)]
    e[0] = g[0].copy()
    if k == len(phis) - 1:
        for n in range(1, N + 1):
            e[n] = phis[k](e[n - 1]) + g[n]
        return e
    _relax(phis[k], e, g, c, relax)
    r = _residual(phis[k], e, g, c)
    ec = _cycle(phis, k + 1, r, c, relax)
    for m in range(N // c + 1):
        e[c * m] = e[c * m] + ec[m]
    _f_relax(phis[k], e, g, c)
    return e


def solve(phis, u0, N: int, c: int, tol: float, maxit: int, relax: str = "FCF",
          history: list | None = None, all_points: list | None = None):
    """MGRIT on level 0 with propagators phis[0..levels-1].
    Returns (u_N, iterations, converged); `all_points`, if given, receives
    the level-0 iterate u_0..u_N at return."""
    if N % (c ** (len(phis) - 1)) != 0:
        raise ValueError("N must be divisible by c^(levels-1)")
    u0 = np.asarray(u0, dtype=np.float64)
    g = [u0.copy()] + [np.zeros_like(u0) for _ in range(N)]
    u = [u0.copy() for _ in range(N + 1)]
    if len(phis) == 1:
        for n in range(1, N + 1):
            u[n] = phis[0](u[n - 1])
        return u[N], 0, True
    for it in range(1, maxit + 1):
        _relax(phis[0], u, g, c, relax)
        r = _residual(phis[0], u, g, c)
        norm = max(np.linalg.norm(rm) for rm in r[1:])
        if history is not None:
            history.append(norm)
        if norm <= tol:
            if all_points is not None:
                all_points.extend(u)
            return u[N], it, True
        ec = _cycle(phis, 1, r, c, relax)
        for m in range(N // c + 1):
            u[c * m] = u[c * m] + ec[m]
    if all_points is not None:
        all_points.extend(u)
    return u[N], maxit, False
