"""Exact law of the linear SDE dX = theta X dt + sigma dW of Section 4.4:
from a Gaussian start N(M, C) the density stays Gaussian with

    mean(t) = e^{theta t} M
    cov(t)  = e^{theta t} C e^{theta^T t} + int_0^t e^{theta s} H e^{theta^T s} ds,

H = 2 sigma D sigma^T (the paper prints the mean as e^{sigma t} X_0; the
drift matrix is meant). The integral is taken from one matrix exponential
of the block matrix [[-theta, H], [0, theta^T]] (Van Loan, 1978): with
E = expm(block t) = [[E11, E12], [0, E22]], E22 = e^{theta^T t} and the
integral equals E22^T E12. scipy's expm is the library primitive.

Pinned by tests/test_oracle_sde.py: the moments satisfy their ODEs
d mean/dt = theta mean and d cov/dt = theta cov + cov theta^T + H (central
differences), and the discrete Fokker-Planck solution's moments approach
them under refinement.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def moments(theta, H, M, C, t: float):
    theta = np.asarray(theta, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    d = theta.shape[0]
    E = expm(theta * t)
    mean = E @ np.asarray(M, dtype=np.float64)
    blk = np.zeros((2 * d, 2 * d))
    blk[:d, :d] = -theta
    blk[:d, d:] = H
    blk[d:, d:] = theta.T
    F = expm(blk * t)
    integral = F[d:, d:].T @ F[:d, d:]
    cov = E @ np.asarray(C, dtype=np.float64) @ E.T + integral
    return mean, cov


def density(X: np.ndarray, mean, cov) -> np.ndarray:
    d = X.shape[1]
    Z = X - mean
    P = np.linalg.inv(cov)
    q = np.einsum("ni,ij,nj->n", Z, P, Z)
    return np.exp(-0.5 * q) / np.sqrt((2 * np.pi) ** d * np.linalg.det(cov))
