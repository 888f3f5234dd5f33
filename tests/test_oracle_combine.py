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


# ------------------------------------------------------- hierarchical basis
def _level_of(J, li):
    # level at which node index J (0 < J < 2^li) first appears
    tz = (J & -J).bit_length() - 1
    return li - tz


@pytest.mark.parametrize("l", [(5,), (3, 4), (2, 3, 4), (4, 1, 2)])
def test_hierarchical_surplus_closed_form(l):
    # f = prod (x_i - lo_i)(hi_i - x_i) has f_i'' = -2 on every axis, so the
    # 1-D surplus f(x) - (f(x-h) + f(x+h))/2 at a level-k node is h_k^2 and
    # the tensor surplus is the product over axes
    p = make("heat3d", d=len(l), n=max(l) + 1)
    p["lo"] = [-0.5, 0.25, 1.0][: len(l)]
    p["hi"] = [1.5, 2.25, 1.75][: len(l)]
    lo, hi = np.asarray(p["lo"]), np.asarray(p["hi"])
    X = grids.coordinates(p, l)
    u = np.prod((X - lo) * (hi - X), axis=1)
    uh = combine.hierarchize(p, l, u)
    J = [np.arange(1, 2 ** li) for li in l]
    mesh = np.meshgrid(*J, indexing="ij")
    want = np.ones(mesh[0].size)
    for i, li in enumerate(l):
        k = np.array([_level_of(int(j), li) for j in mesh[i].reshape(-1)])
        want *= ((hi[i] - lo[i]) * 2.0 ** (-k)) ** 2
    assert np.abs(uh - want).max() <= 1e-14 * np.abs(want).max() * 16


def test_hierarchical_lattice_linear_has_level0_only():
    # on a lattice axis the interpolant is 0 at hi; (hi - x) is reproduced by
    # the level-0 function alone: one coefficient hi - lo at the origin
    p = make("cme5d", d=2, n=4, hi=[16.0, 16.0])
    for l in [(4, 2), (1, 3), (3, 3)]:
        X = grids.coordinates(p, l)
        u = np.prod(16.0 - X, axis=1)
        uh = combine.hierarchize(p, l, u)
        assert abs(uh[0] - 256.0) <= 1e-12
        assert np.abs(uh[1:]).max() <= 1e-12


@pytest.mark.parametrize("name,d,n", [("heat3d", 3, 5), ("cme5d", 3, 4), ("ou4d", 2, 6)])
def test_hierarchize_roundtrip(name, d, n):
    p = make(name, d=d, n=n)
    rng = np.random.default_rng(4)
    for (l, _, _) in index_set.combination_grids(d, n, 1)[:6]:
        u = rng.standard_normal(int(np.prod(grids.shape(p, l))))
        back = combine.dehierarchize(p, l, combine.hierarchize(p, l, u))
        assert np.abs(back - u).max() <= 1e-13


@pytest.mark.parametrize("name,d,n", [("heat3d", 3, 5), ("cme5d", 3, 4), ("heat2d", 2, 6),
                                      ("varcoef6d", 4, 4)])
def test_recombine_hier_equals_direct_projection(name, d, n):
    # Q = H^-1 Qbar H equals combine-then-take-node-values (Section 2.2.2)
    p = make(name, d=d, n=n)
    gl = index_set.combination_grids(d, n, 1)
    rng = np.random.default_rng(5)
    states = [rng.standard_normal(int(np.prod(grids.shape(p, l)))) for (l, _, _) in gl]
    a = combine.recombine_hier(p, gl, states)
    b = combine.project(p, gl, states)
    scale = sum(abs(c) for (_, _, c) in gl)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-13 * scale
