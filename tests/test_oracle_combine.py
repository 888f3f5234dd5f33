"""Pins of the oracle's combination (interpolation properties of the
sparse-grid combination)."""
import math

import numpy as np
import pytest

from oracle import combine, grids, index_set
from workloads import make, targets


def _smooth(X, lo, hi):
    # an arbitrary smooth function that vanishes on the Dirichlet boundary
    t = (X - lo) / (hi - lo)
    return np.prod(np.sin(math.pi * t) * np.exp(0.3 * t + np.cos(2.1 * t)), axis=1) + \
        0.5 * np.prod(np.sin(2 * math.pi * t), axis=1)


@pytest.mark.parametrize("name,d,n", [("heat2d", 2, 5), ("heat3d", 3, 5), ("ou4d", 4, 4),
                                      ("cme5d", 3, 4), ("heat2d", 1, 6)])
def test_combination_interpolates_at_component_nodes(name, d, n):
    # The combination of the interpolants of one function sampled on every
    # component grid equals the sparse-grid interpolant, which interpolates
    # at all sparse-grid nodes -- in particular at every component node.
    p = make(name, d=d, n=n)
    lo, hi = np.asarray(p["lo"]), np.asarray(p["hi"])
    if p["op"] == "cme":
        f = lambda X: np.prod(np.exp(-0.05 * (X - lo)), axis=1) * (1 + 0.1 * np.sum(X, axis=1))
    else:
        f = lambda X: _smooth(X, lo, hi)
    gl = index_set.combination_grids(d, n, 1)
    states = [f(grids.coordinates(p, l)) for (l, _, _) in gl]
    scale = sum(abs(c) for (_, _, c) in gl)
    for (l, _, _) in gl:
        X = grids.coordinates(p, l)
        got = combine.combine_at(p, gl, states, X)
        assert np.abs(got - f(X)).max() <= 64 * scale * 2.3e-16 * max(1, np.abs(f(X)).max())


@pytest.mark.parametrize("d,n", [(2, 6), (3, 5), (4, 4)])
def test_combination_reproduces_one_coordinate_functions(d, n):
    # f(x) = g(x_1) prod_{j>=2} phi(x_j), phi the level-1 hat, lies in V_m
    # along axes 2..d for every m; the combination coefficients of all grids
    # with the same m_1 add up to 1 for m_1 = n and to 0 otherwise, so the
    # result is (I_n g)(x_1) prod phi(x_j), with I_n the level-n 1-D
    # piecewise linear interpolant of g.
    p = make("heat2d", d=d, n=n)
    g = lambda x: np.sin(3.0 * x) * x * (1 - x) + x ** 2 * (1 - x)
    hat = lambda x: 1.0 - np.abs(2.0 * x - 1.0)

    def f(X):
        return g(X[:, 0]) * np.prod(hat(X[:, 1:]), axis=1)

    gl = index_set.combination_grids(d, n, 1)
    states = [f(grids.coordinates(p, l)) for (l, _, _) in gl]
    P = targets(p, 500, seed=4)
    xs = np.linspace(0, 1, 2 ** n + 1)
    ref = np.interp(P[:, 0], xs, g(xs) * (xs > 0) * (xs < 1)) * np.prod(hat(P[:, 1:]), axis=1)
    got = combine.combine_at(p, gl, states, P)
    assert np.abs(got - ref).max() <= 1e-13


def test_combination_exact_on_common_space():
    # prod phi(x_j) (level-1 hats) lies in every component space, and the
    # coefficients sum to 1: the combination reproduces it at any point.
    p = make("heat3d", n=6)
    hat = lambda X: np.prod(1.0 - np.abs(2.0 * X - 1.0), axis=1)
    gl = index_set.combination_grids(3, 6, 1)
    states = [hat(grids.coordinates(p, l)) for (l, _, _) in gl]
    P = targets(p, 1000, seed=5)
    assert np.abs(combine.combine_at(p, gl, states, P) - hat(P)).max() <= 1e-13


def test_interpolant_between_nodes_and_boundary():
    # 1-D spot values of I_l: linear between nodes, zero at the Dirichlet ends.
    p = make("heat2d", d=1, n=3)
    u = np.array([1.0, 2.0, 4.0])      # level 2: nodes 0.25, 0.5, 0.75
    pts = np.array([[0.0], [0.125], [0.375], [0.6], [0.875], [1.0]])
    got = combine.interpolate(p, (2,), u, pts)
    assert np.allclose(got, [0.0, 0.5, 1.5, 2.8, 2.0, 0.0], atol=1e-15)
    # lattice axis: nodes at 0, 32 (level 1 of 0..63); zero node at 64
    q = make("cme5d", d=1)
    got = combine.interpolate(q, (1,), np.array([3.0, 5.0]), np.array([[0.0], [16.0], [48.0], [63.0]]))
    assert np.allclose(got, [3.0, 4.0, 2.5, 5.0 / 32], atol=1e-15)
