"""Pins of the oracle's recombination blocks (Algorithm 1 with s > 1):
solve.component_states against the composition of its parts, each pinned
on its own -- time-sequential stepping (oracle.propagate) and the
hierarchical combine-then-project (oracle.combine.recombine_hier, which is
pinned against the direct projection and the closed-form surpluses)."""
import numpy as np
import pytest

from oracle import combine, grids, propagate, solve
from workloads import make


def _composed(p, s):
    """s blocks: march N/s steps on every grid, project through the
    hierarchical basis between blocks (not after the last), with the
    forcing clock of block k starting at t0 + k N/s dt."""
    gl = solve.grid_list(p)
    dt = propagate.step_size(p, 0)
    nb = p["nsteps"] // s
    u = [grids.initial_value(p, l) for (l, _, _) in gl]
    for k in range(s):
        if k > 0:
            u = combine.recombine_hier(p, gl, u)
        u = [propagate.march(p, l, x, nb, dt, t_start=p["t0"] + k * nb * dt)
             for (l, _, _), x in zip(gl, u)]
    return u


@pytest.mark.parametrize("name,kw,s", [
    ("heat2d", dict(n=5), 2),
    ("heat2d", dict(n=5), 4),
    ("ou4d", dict(d=2, n=5), 2),
    ("cme5d", dict(d=2, n=4, lo=[0.0, 0.0], hi=[16.0, 16.0]), 2),
    ("heat_mms", dict(d=2, n=5), 2),   # forced: the clock continues across blocks
    ("heat_mms", dict(d=3, n=4), 4),
])
def test_blocks_equal_their_composition(name, kw, s):
    p = make(name, **kw)
    p.update(nsteps=8, t1=p["t0"] + 8 * (p["t1"] - p["t0"]) / p["nsteps"], nrecomb=s)
    got = solve.component_states(p)
    want = _composed(p, s)
    scale = max(np.abs(x).max() for x in want)
    for a, b in zip(got, want):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * scale)


def test_projection_is_not_applied_after_the_last_block():
    # a projection after the last block would change the states of the
    # coarse grids (their values become the combined solution there)
    p = make("heat2d", n=5)
    p.update(nsteps=8, t1=0.1 * 8 / 64, nrecomb=2)
    gl = solve.grid_list(p)
    got = solve.component_states(p)
    proj = combine.recombine_hier(p, gl, got)
    assert max(np.abs(a - b).max() for a, b in zip(got, proj)) > 1e-6


def test_forcing_clock_matters():
    # restarting the forcing clock at t0 in the second block gives another
    # result: the pin above separates the two
    p = make("heat_mms", d=2, n=5)
    p.update(nsteps=8, t1=1.0, nrecomb=2)
    gl = solve.grid_list(p)
    dt = propagate.step_size(p, 0)
    u = [propagate.march(p, l, grids.initial_value(p, l), 4, dt) for (l, _, _) in gl]
    u = combine.recombine_hier(p, gl, u)
    wrong = [propagate.march(p, l, x, 4, dt, t_start=p["t0"]) for (l, _, _), x in zip(gl, u)]
    got = solve.component_states(p)
    assert max(np.abs(a - b).max() for a, b in zip(got, wrong)) > 1e-6


def test_one_dimension_one_grid_blocks_are_plain_stepping():
    # d = 1: one component grid with coefficient 1, so combine-then-project
    # is the identity and s = 2 equals s = 1
    p = make("heat2d", d=1, n=6)
    p.update(nsteps=8, t1=0.1 * 8 / 64)
    one = solve.component_states(dict(p, nrecomb=1))
    two = solve.component_states(dict(p, nrecomb=2))
    assert len(one) == 1
    np.testing.assert_allclose(two[0], one[0], rtol=0, atol=1e-15 * np.abs(one[0]).max())
