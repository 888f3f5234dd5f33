"""Pins of the oracle's spatial operators against closed forms, invariants and
consistency with the continuous operators."""
import math

import numpy as np
import pytest

from oracle import grids, operators
from workloads import make


def _heat(d, n=6):
    return make("heat2d", n=n, d=d)


@pytest.mark.parametrize("l,k", [((3, 2), (1, 1)), ((4, 1), (3, 1)), ((2, 5), (2, 7)),
                                 ((1, 1, 3), (1, 1, 2)), ((3, 2, 2), (5, 1, 3)), ((2, 3), (4, 8))])
def test_heat_sine_modes_are_eigenvectors(l, k):
    # Discrete sine modes sin(pi k x) are eigenvectors of the 5/7-point
    # Laplacian with eigenvalue sum_i 4 h_i^-2 sin^2(pi k_i h_i / 2); a mode
    # aliased to zero on a coarse axis gives the zero vector.
    p = _heat(len(l))
    X = grids.coordinates(p, l)
    v = np.prod([np.sin(math.pi * k[i] * X[:, i]) for i in range(len(l))], axis=0)
    lam = sum(4.0 * 4 ** l[i] * math.sin(math.pi * k[i] / 2 ** l[i] / 2) ** 2 for i in range(len(l)))
    L = operators.matrix(p, l)
    scale = max(1.0, lam) * max(1.0, np.abs(v).max())
    assert np.abs(L @ v - lam * v).max() <= 1e-12 * scale


def test_varcoef_reduces_to_heat_and_is_symmetric():
    p = make("varcoef6d", d=3, n=5)
    for l in [(2, 2, 3), (1, 4, 2), (3, 3, 1)]:
        Lv = operators.matrix(p, l)
        assert abs(Lv - Lv.T).max() <= 1e-12 * abs(Lv).max()
        p0 = dict(p, amp=0.0)
        Lh = operators.matrix(dict(p, op="heat"), l)
        assert abs(operators.matrix(p0, l) - Lh).max() <= 1e-12 * abs(Lh).max()


def _div_a_grad(X, amp):
    # -div(a grad u) for u = prod sin(pi x_i), a = 1 + amp prod sin(2 pi x_k),
    # written from the product rule: -(a Lap u + grad a . grad u).
    d = X.shape[1]
    s = np.sin(math.pi * X)
    c = np.cos(math.pi * X)
    s2 = np.sin(2 * math.pi * X)
    c2 = np.cos(2 * math.pi * X)
    u = np.prod(s, axis=1)
    a = 1 + amp * np.prod(s2, axis=1)
    lap = -d * math.pi ** 2 * u
    ga_gu = np.zeros(X.shape[0])
    for i in range(d):
        others = [k for k in range(d) if k != i]
        da = amp * 2 * math.pi * c2[:, i] * np.prod(s2[:, others], axis=1)
        du = math.pi * c[:, i] * np.prod(s[:, others], axis=1)
        ga_gu += da * du
    return -(a * lap + ga_gu), u


def test_varcoef_second_order_consistent():
    p = make("varcoef6d", d=2, n=8)
    errs = []
    for lev in (4, 5, 6):
        l = (lev, lev)
        X = grids.coordinates(p, l)
        exact, u = _div_a_grad(X, 0.5)
        errs.append(np.abs(operators.matrix(p, l) @ u - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def _ou(d=2, n=6):
    p = make("ou4d", d=d, n=n)
    return p


def test_ou_column_sums_and_sign_pattern():
    p = _ou(2)
    for l in [(4, 3), (5, 5), (2, 6)]:
        L = operators.matrix(p, l).toarray()
        off = L - np.diag(np.diag(L))
        assert (off <= 0).all() and (np.diag(L) > 0).all()
        shp = grids.shape(p, l)
        idx = np.arange(L.shape[0]).reshape(shp)
        inner = idx[tuple(slice(1, -1) for _ in shp)].reshape(-1)
        colsum = L.sum(axis=0)
        assert np.abs(colsum[inner]).max() <= 1e-10 * np.abs(L).max()
        # boundary-adjacent columns lose mass to the zero ghosts (diffusion only)
        edge = np.setdiff1d(np.arange(L.shape[0]), inner)
        assert (colsum[edge] > 0).all()


def test_ou_first_order_consistent():
    # -L u approximates d/dx(theta x u) + (sigma^2/2) u'' for a Gaussian bump
    # (1-D); donor-cell fluxes make the error first order in h.
    p = make("ou4d", d=1, n=12)
    theta, D = p["theta"][0], 0.5 * p["sigma"] ** 2
    errs = []
    for lev in (7, 8, 9):
        x = grids.axis_nodes(p, (lev,), 0)
        u = np.exp(-(x - 0.3) ** 2)
        du = -2 * (x - 0.3) * u
        d2u = (4 * (x - 0.3) ** 2 - 2) * u
        exact = theta * u + theta * x * du + D * d2u
        mask = np.abs(x) < 4
        errs.append(np.abs((-(operators.matrix(p, (lev,)) @ u) - exact)[mask]).max())
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4, errs


def test_cme_conservative_and_m_matrix():
    p = make("cme5d", d=3)
    for l in [(2, 3, 1), (6, 1, 1), (3, 3, 2)]:
        L = operators.matrix(p, l).toarray()
        assert np.abs(L.sum(axis=0)).max() <= 1e-12 * np.abs(L).max()
        off = L - np.diag(np.diag(L))
        assert (off <= 0).all() and (np.diag(L) >= 0).all()


@pytest.mark.parametrize("lev", [6, 4, 2, 1])
def test_cme_stationary_truncated_poisson(lev):
    # A birth-death chain with birth rate k/h and death rate gamma x / h
    # (x = j h) satisfies detailed balance with pi(j) ~ (k / (gamma h))^j / j!
    # on j = 0..2^lev - 1: the truncated Poisson law of mean k / (gamma h).
    p = make("cme5d", d=1)
    k, g = p["k"][0], p["gamma"][0]
    h = 64 / 2 ** lev
    lam = k / (g * h)
    j = np.arange(2 ** lev)
    logpi = j * math.log(lam) - np.array([math.lgamma(v + 1) for v in j])
    pi = np.exp(logpi - logpi.max())
    pi /= pi.sum()
    L = operators.matrix(p, (lev,))
    assert np.abs(L @ pi).max() <= 1e-12 * np.abs(L).max()
