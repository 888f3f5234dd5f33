"""Manufactured-solution heat problem of Section 4.2 (heat equation in
higher dimensions): on Omega = [0,1]^d,

    u*(x, t) = sqrt(|x|^2 + t^2) e^-t prod_i sin(pi x_i),

which vanishes on the boundary, and the forcing f = du*/dt - Laplace(u*)
that makes u* the exact solution. The derivatives are written out here by
the product and chain rules (r = sqrt(|x|^2 + t^2), S = prod_i sin(pi x_i),
S_i = the product without factor i):

    du*/dt     = e^-t S (t / r - r)
    Laplace u* = e^-t [ S (d / r - |x|^2 / r^3)
                        + (2 pi / r) sum_i x_i cos(pi x_i) S_i
                        - d pi^2 r S ]

The backward-Euler step with forcing (Section 2, time propagation) is
u_n = (I + dt L)^-1 (u_{n-1} + dt f(., t_n)).

Pinned by tests/test_oracle_manufactured.py: f against central finite
differences of u* in t and in every x_i, and the discrete solution
converging to u* under refinement.
"""
from __future__ import annotations

import numpy as np


def u_star(X: np.ndarray, t: float) -> np.ndarray:
    """u*(x, t) at the rows of X (shape (M, d))."""
    r = np.sqrt(np.sum(X * X, axis=1) + t * t)
    return r * np.exp(-t) * np.prod(np.sin(np.pi * X), axis=1)


def forcing(X: np.ndarray, t: float) -> np.ndarray:
    """f = du*/dt - Laplace(u*) at the rows of X."""
    d = X.shape[1]
    x2 = np.sum(X * X, axis=1)
    r = np.sqrt(x2 + t * t)
    sn = np.sin(np.pi * X)
    S = np.prod(sn, axis=1)
    cross = np.zeros(X.shape[0])
    for i in range(d):
        others = np.prod(np.delete(sn, i, axis=1), axis=1) if d > 1 else np.ones(X.shape[0])
        cross += X[:, i] * np.cos(np.pi * X[:, i]) * others
    dudt = S * (t / r - r)
    lap = S * (d / r - x2 / r ** 3) + (2.0 * np.pi / r) * cross - d * np.pi ** 2 * r * S
    return np.exp(-t) * (dudt - lap)


def is_manufactured(prob) -> bool:
    return prob.get("manufactured") == "heat"
