"""Pins of the oracle's backward-Euler propagator and time stepping."""
import math

import numpy as np
import pytest

from oracle import grids, krylov, operators, propagate, solve
from workloads import make


def heat_closed_form(p, l, nsteps, dt):
    """Exact discrete solution of backward Euler for a sum of sine modes:
    every mode is damped by (1 + dt lambda)^-1 per step."""
    X = grids.coordinates(p, l)
    out = np.zeros(X.shape[0])
    modes = p.get("modes", [[1] * p["d"]])
    for w, kv in zip(p["ic_w"], modes):
        lam = sum(4.0 * 4 ** l[i] * math.sin(math.pi * kv[i] / 2 ** l[i] / 2) ** 2
                  for i in range(len(l)))
        v = np.prod([np.sin(math.pi * kv[i] * X[:, i]) for i in range(len(l))], axis=0)
        out += w * (1.0 + dt * lam) ** (-nsteps) * v
    return out


@pytest.mark.parametrize("name,grid_idx", [("heat2d", None), ("heat3d", [0, 5, 44, 45, 80, 108])])
def test_heat_components_match_closed_form(name, grid_idx):
    p = make(name)
    gl = solve.grid_list(p)
    sel = range(len(gl)) if grid_idx is None else grid_idx
    states = solve.component_states(p, sel)
    dt = propagate.step_size(p)
    for g, u in zip(sel, states):
        ref = heat_closed_form(p, gl[g][0], p["nsteps"], dt)
        # rounding grows with the number of steps; a wrong term is O(1)
        assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max() + 1e-15


@pytest.mark.parametrize("name,l", [("heat3d", (4, 4, 3)), ("heat3d", (9, 1, 1)),
                                    ("varcoef6d", (2, 2, 1, 1, 2, 1)), ("ou4d", (3, 3, 3, 2)),
                                    ("ou4d", (8, 1, 1, 1)), ("cme5d", (2, 2, 1, 1, 1)),
                                    ("cme5d", (6, 1, 1, 1, 1))])
def test_lu_agrees_with_krylov(name, l):
    p = make(name)
    dt = propagate.step_size(p, 1)
    A = operators.system_matrix(p, l, dt)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    x_lu = propagate.Propagator(p, l, dt)(b)
    solver = krylov.cg if operators.is_symmetric(p) else krylov.bicgstab
    x_kr, _ = solver(A, b, tol=1e-14)
    assert np.linalg.norm(x_lu - x_kr) <= 1e-11 * np.linalg.norm(x_lu)
    assert np.linalg.norm(A @ x_lu - b) <= 1e-13 * np.linalg.norm(b) * max(1, abs(A).max())


@pytest.mark.parametrize("l", [(2, 3, 1), (1, 4, 2), (3, 3, 3)])
def test_cme_marginal_identity(l):
    # For a Kronecker sum of conservative generators, summing the d-D
    # backward-Euler solution over all axes but i gives exactly the 1-D
    # backward-Euler solution on axis i (times the sums of the other initial
    # factors).
    p = make("cme5d", d=3)
    rng = np.random.default_rng(3)
    # product initial value with random positive factors
    f = rng.uniform(0.1, 1.0, size=(1, 3, 2 ** p["n"] + 1))
    p["ic_f"] = f
    dt, N = 0.05, 7
    u = propagate.march(p, l, grids.initial_value(p, l), N, dt).reshape(grids.shape(p, l))
    for i in range(3):
        p1 = make("cme5d", d=1)
        p1.update(k=[p["k"][i]], gamma=[p["gamma"][i]], ic_f=f[:, i:i + 1, :])
        u1 = propagate.march(p1, (l[i],), grids.initial_value(p1, (l[i],)), N, dt)
        others = 1.0
        for j in range(3):
            if j != i:
                others *= grids.initial_value(dict(p1, ic_f=f[:, j:j + 1, :]), (l[j],)).sum()
        marg = u.sum(axis=tuple(j for j in range(3) if j != i))
        assert np.abs(marg - others * u1).max() <= 1e-12 * np.abs(marg).max()


def test_cme_unit_spacing_chain_tends_to_poisson():
    # The lattice chain at spacing 1 is the immigration-death master equation;
    # from state 0 its exact law at time t is Poisson with mean
    # (k / gamma)(1 - exp(-gamma t)) (truncation at 63 is negligible). Backward
    # Euler is first order in dt: halving dt halves the error.
    p = make("cme5d", d=1)
    k, g, T = p["k"][0], p["gamma"][0], 2.0
    mean = k / g * (1 - math.exp(-g * T))
    j = np.arange(64)
    pmf = np.exp(j * math.log(mean) - mean - np.array([math.lgamma(v + 1) for v in j]))
    errs = []
    for N in (256, 512, 1024):
        u = propagate.march(p, (6,), grids.initial_value(p, (6,)), N, T / N)
        errs.append(np.abs(u - pmf).max())
    assert errs[0] < 5e-3
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs


def test_ou_moments_tend_to_gaussian_law():
    # 1-D OU density: mean mu0 exp(-theta t), variance
    # v0 exp(-2 theta t) + sigma^2 (1 - exp(-2 theta t)) / (2 theta).
    # Upwinding and backward Euler are first order; the error must shrink.
    p = make("ou4d", d=1, n=12)
    theta, mu0, v0, T = p["theta"][0], p["mu0"][0], p["var0"], 1.0
    m_ex = mu0 * math.exp(-theta * T)
    v_ex = v0 * math.exp(-2 * theta * T) + (1 - math.exp(-2 * theta * T)) / (2 * theta)
    errs = []
    for lev, N in ((8, 128), (9, 256), (10, 512)):
        x = grids.axis_nodes(p, (lev,), 0)
        u = propagate.march(p, (lev,), grids.initial_value(p, (lev,)), N, T / N)
        mass = u.sum()
        m = (x * u).sum() / mass
        v = ((x - m) ** 2 * u).sum() / mass
        errs.append(abs(m - m_ex) + abs(v - v_ex))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 2e-2, errs
