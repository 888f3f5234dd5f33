"""Textbook Krylov solvers (Section 4.1: CG for symmetric operators,
BiCGStab for non-symmetric ones), plain and preconditioned.

Used to cross-check the direct solves of oracle.propagate and to count the
iterations of the preconditioned solvers; each follows the standard
algorithm statement (Hestenes-Stiefel CG and its preconditioned form;
van der Vorst's BiCGStab, preconditioned from the right) with the stopping
test ||b - A x||_2 <= tol ||b||_2 on the recursively updated residual.

Pinned by tests/test_oracle_propagate.py: both plain solvers agree with the
sparse LU solve to 1e-11 on every operator kind; by
tests/test_oracle_schwarz.py: with the identity as preconditioner the
preconditioned solvers take the plain ones' iterations, and with the exact
inverse they stop after one iteration.
"""
from __future__ import annotations

import numpy as np


def cg(A, b, x0=None, tol=1e-13, maxit=100000):
    x = np.array(b if x0 is None else x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0
    r = b - A @ x
    p = r.copy()
    rr = r @ r
    for it in range(maxit):
        if np.sqrt(rr) <= tol * bnorm:
            return x, it
        q = A @ p
        alpha = rr / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise RuntimeError("CG did not converge")


def bicgstab(A, b, x0=None, tol=1e-13, maxit=100000):
    x = np.array(b if x0 is None else x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0
    r = b - A @ x
    rhat = r.copy()
    rho = alpha = omega = 1.0
    v = np.zeros_like(x)
    p = np.zeros_like(x)
    for it in range(maxit):
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it
        rho_new = rhat @ r
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A @ p
        alpha = rho_new / (rhat @ v)
        s = r - alpha * v
        t = A @ s
        tt = t @ t
        omega = (t @ s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
    raise RuntimeError("BiCGStab did not converge")


def pcg(A, b, M, x0=None, tol=1e-13, maxit=100000):
    """CG preconditioned by the matrix M (an approximation of A^-1)."""
    x = np.zeros_like(b, dtype=np.float64) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0
    r = b - A @ x
    z = M @ r
    p = z.copy()
    rz = r @ z
    for it in range(maxit):
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = M @ r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError("PCG did not converge")


def pbicgstab(A, b, M, x0=None, tol=1e-13, maxit=100000):
    """BiCGStab preconditioned from the right by the matrix M: the iteration
    of bicgstab on A M with x = M y."""
    x = np.zeros_like(b, dtype=np.float64) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(x), 0
    r = b - A @ x
    rhat = r.copy()
    rho = alpha = omega = 1.0
    v = np.zeros_like(x)
    p = np.zeros_like(x)
    for it in range(maxit):
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it
        rho_new = rhat @ r
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = M @ p
        v = A @ ph
        alpha = rho_new / (rhat @ v)
        s = r - alpha * v
        sh = M @ s
        t = A @ sh
        tt = t @ t
        omega = (t @ s) / tt if tt > 0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho = rho_new
    raise RuntimeError("preconditioned BiCGStab did not converge")
