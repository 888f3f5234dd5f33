"""Pins of the manufactured heat problem (Section 4.2): the forcing against
finite differences of u*, and the oracle's discrete solution converging to
u* under refinement."""
import numpy as np
import pytest

from oracle import combine, grids, manufactured, solve
from workloads import make


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_forcing_matches_finite_differences(d):
    rng = np.random.default_rng(d)
    X = rng.uniform(0.05, 0.95, size=(40, d))
    for t in [0.05, 0.4, 1.0]:
        h = 1e-4
        dudt = (manufactured.u_star(X, t + h) - manufactured.u_star(X, t - h)) / (2 * h)
        lap = np.zeros(X.shape[0])
        for i in range(d):
            E = np.zeros(d)
            E[i] = h
            lap += (manufactured.u_star(X + E, t) - 2 * manufactured.u_star(X, t)
                    + manufactured.u_star(X - E, t)) / h ** 2
        f = manufactured.forcing(X, t)
        scale = np.abs(f).max()
        assert np.abs(f - (dudt - lap)).max() <= 1e-5 * scale


def test_exact_solution_vanishes_on_boundary():
    X = np.array([[0.0, 0.3], [1.0, 0.7], [0.4, 0.0], [0.2, 1.0]])
    assert np.abs(manufactured.u_star(X, 0.5)).max() <= 1e-15


def test_discrete_solution_converges_to_exact():
    # combination solution at T against u*(., T) at seeded points: the error
    # falls by about 4 when h halves and dt quarters (O(h^2) + O(dt))
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.1, 0.9, size=(200, 2))
    errs = []
    for n, N in [(4, 8), (5, 32), (6, 128)]:
        p = make("heat_mms", d=2, n=n, nsteps=N, t1=0.5)
        gl = solve.grid_list(p)
        states = solve.component_states(p)
        got = combine.combine_at(p, gl, states, pts)
        errs.append(np.abs(got - manufactured.u_star(pts, 0.5)).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_initial_value_is_exact_solution_at_t0():
    p = make("heat_mms", d=3, n=4)
    for (l, _, _) in solve.grid_list(p)[:5]:
        X = grids.coordinates(p, l)
        assert np.array_equal(grids.initial_value(p, l), manufactured.u_star(X, 0.0))
