"""Pins of the two-level Schwarz preconditioner of the spatial solver
(Section 2.1.2) and of the preconditioned Krylov solvers (Section 4.1)."""
import itertools
import math

import numpy as np
import pytest

from oracle import krylov, operators, schwarz
from workloads import make


@pytest.mark.parametrize("d,bits", [(1, 3), (2, 1), (2, 3), (3, 2), (3, 3), (4, 2)])
def test_hilbert_curve_is_a_lattice_walk(d, bits):
    # the curve visits every point of the 2^bits lattice once, and
    # consecutive points differ by one in exactly one coordinate (a Morton
    # or row-major order fails the second test)
    side = 2 ** bits
    pts = list(itertools.product(range(side), repeat=d))
    keys = [schwarz.hilbert_index(p, bits) for p in pts]
    assert sorted(keys) == list(range(side ** d))
    walk = np.array([p for _, p in sorted(zip(keys, pts))])
    steps = np.abs(np.diff(walk, axis=0))
    assert (steps.sum(axis=1) == 1).all()
    # starts at the origin
    assert tuple(walk[0]) == (0,) * d


def test_curve_order_of_an_anisotropic_grid():
    # virtual nodes: the unknowns of l = (2, 3) sit at even lattice columns
    # of the level-3 lattice; the order is a permutation, and consecutive
    # unknowns stay close (at most two lattice steps apart here, the width
    # of the virtual gap)
    p = make("heat2d")
    l = (2, 3)
    C = schwarz.lattice_coordinates(p, l)
    assert set(C[:, 0]) == {2, 4, 6} and set(C[:, 1]) == set(range(1, 8))
    order = schwarz.curve_order(p, l)
    assert sorted(order) == list(range(len(C)))
    gaps = np.abs(np.diff(C[order], axis=0)).sum(axis=1)
    assert gaps.max() <= 4 and np.median(gaps) <= 2


@pytest.mark.parametrize("N_l,S", [((5, 4), 3), ((4, 4), 4), ((6, 3), 4), ((3, 3, 3), 5)])
def test_partition_sizes_and_overlap(N_l, S):
    # Section 2.1.2: P = ceil(N / 2^S) subdomains, N - P w of them of size
    # w + 1 and the others of size w = floor(N / P); with gamma = 1/2 the
    # points within floor(w / 2) of an interior boundary lie in two extended
    # subdomains, no point in more, and subdomains two apart are disjoint
    p = make("heat2d") if len(N_l) == 2 else make("heat3d")
    dec = schwarz.Decomposition(p, N_l, S)
    N = dec.N
    P = math.ceil(N / 2 ** S)
    assert dec.P == P
    sizes = [b - a for a, b in dec.disjoint]
    w = N // P
    assert sizes.count(w + 1) == N - P * w and sizes.count(w) == P - (N - P * w)
    assert sum(sizes) == N
    assert dec.multiplicity.max() <= 2 and dec.multiplicity.min() >= 1
    if P > 1:
        ov = w // 2
        for a, _ in dec.disjoint[1:]:
            assert (dec.multiplicity[a - ov:a + ov] == 2).all()
        assert all(om == 0.5 for om in dec.omega)
        for (a0, b0), (a2, b2) in zip(dec.extended, dec.extended[2:]):
            assert b0 <= a2
        if w % 2 == 0:
            assert (dec.multiplicity == 2).sum() == N - 2 * ov
    # coarse blocks partition the curve
    cov = np.zeros(N, dtype=int)
    for a, b in dec.blocks:
        cov[a:b] += 1
    assert (cov == 1).all()


def _spd_case():
    p = make("varcoef6d", d=2, n=5)
    l = (4, 3)
    A = operators.system_matrix(p, l, 0.01).toarray()
    return p, l, A


def test_coarse_projection_identity():
    # F A F = F, hence (I - F A) is a projection
    p, l, A = _spd_case()
    dec = schwarz.Decomposition(p, l, 3)
    F = schwarz.coarse(A, dec)
    assert np.abs(F @ A @ F - F).max() <= 1e-12 * np.abs(F).max()


def test_balanced_is_exact_for_one_subdomain_or_full_coarse_space():
    # one subdomain: C1 = A^-1 and G^T A^-1 G + F = A^-1 - F - F + F A F + F
    # = A^-1 for any coarse space; a coarse space holding every point gives
    # F = A^-1, G = 0
    p, l, A = _spd_case()
    Ainv = np.linalg.inv(A)
    one = schwarz.Decomposition(p, l, 10)
    assert one.P == 1
    np.testing.assert_allclose(schwarz.balanced(A, one), Ainv, atol=1e-12 * np.abs(Ainv).max())
    full = schwarz.Decomposition(p, l, 3, q=10 ** 6)
    assert len(full.blocks) == full.N
    np.testing.assert_allclose(schwarz.balanced(A, full), Ainv, atol=1e-11 * np.abs(Ainv).max())
    # the additive form is not exact for one subdomain: it adds F
    assert np.abs(schwarz.additive(A, one) - Ainv).max() > 1e-3 * np.abs(Ainv).max()


def test_balanced_symmetric_positive_definite():
    p, l, A = _spd_case()
    C = schwarz.balanced(A, schwarz.Decomposition(p, l, 3))
    assert np.abs(C - C.T).max() <= 1e-12 * np.abs(C).max()
    assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0


def test_preconditioned_solvers_reduce_to_plain_and_exact():
    rng = np.random.default_rng(3)
    p, l, A = _spd_case()
    b = rng.standard_normal(A.shape[0])
    I = np.eye(A.shape[0])
    x0, it0 = krylov.cg(A, b, x0=np.zeros_like(b), tol=1e-12)
    x1, it1 = krylov.pcg(A, b, I, tol=1e-12)
    assert it1 == it0 and np.abs(x1 - x0).max() <= 1e-12 * np.abs(x0).max()
    _, it = krylov.pcg(A, b, np.linalg.inv(A), tol=1e-12)
    assert it == 1
    q = make("fp_osc2d", n=5)
    B = operators.system_matrix(q, (3, 4), 0.05).toarray()
    c = rng.standard_normal(B.shape[0])
    y0, jt0 = krylov.bicgstab(B, c, x0=np.zeros_like(c), tol=1e-12)
    y1, jt1 = krylov.pbicgstab(B, c, np.eye(B.shape[0]), tol=1e-12)
    assert jt1 == jt0 and np.abs(y1 - y0).max() <= 1e-10 * np.abs(y0).max()
    _, jt = krylov.pbicgstab(B, c, np.linalg.inv(B), tol=1e-12)
    assert jt == 1


@pytest.mark.parametrize("name,l,dt", [("varcoef6d", (4, 3, 3), 0.01), ("heat3d", (3, 4, 3), 0.02),
                                       ("fp_lin4d", (3, 3, 2, 2), 0.5)])
def test_schwarz_preconditioned_solves(name, l, dt):
    # the preconditioned solvers (balanced with CG, additive with BiCGStab)
    # reach the direct solution, in fewer iterations than without (at steps
    # where the system is far from the identity)
    p = make(name, n=5) if name == "fp_lin4d" else make(name, d=len(l), n=5)
    A = operators.system_matrix(p, l, dt).toarray()
    b = np.random.default_rng(7).standard_normal(A.shape[0])
    x_ref = np.linalg.solve(A, b)
    C = schwarz.preconditioner(p, l, dt, 4)
    if operators.is_symmetric(p):
        x, it = krylov.pcg(A, b, C, tol=1e-12)
        _, it_plain = krylov.cg(A, b, x0=np.zeros_like(b), tol=1e-12)
    else:
        x, it = krylov.pbicgstab(A, b, C, tol=1e-12)
        _, it_plain = krylov.bicgstab(A, b, x0=np.zeros_like(b), tol=1e-12)
    assert np.abs(x - x_ref).max() <= 1e-10 * np.abs(x_ref).max()
    assert it < it_plain
