"""Shared helpers of the GPU parity tests: run the oracle and the HIP path
on the same seeded problem and compare."""
import numpy as np

from oracle import combine, grids, index_set, operators, propagate, solve


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def split(prob, packed):
    """Packed vector -> list of per-grid arrays (canonical order)."""
    off = solve.offsets(prob)
    return [packed[off[g]:off[g + 1]] for g in range(len(off) - 1)]


def oracle_apply(prob, x_packed, level=0):
    gl = solve.grid_list(prob)
    dt = propagate.step_size(prob, level)
    out = []
    for (l, _, _), x in zip(gl, split(prob, x_packed)):
        out.append(operators.system_matrix(prob, l, dt) @ x)
    return np.concatenate(out)


def oracle_abs_apply(prob, x_packed, level=0):
    """|A| |x| per row: the rounding scale of a matrix-vector product."""
    gl = solve.grid_list(prob)
    dt = propagate.step_size(prob, level)
    out = []
    for (l, _, _), x in zip(gl, split(prob, x_packed)):
        out.append(abs(operators.system_matrix(prob, l, dt)) @ np.abs(x))
    return np.concatenate(out)


def oracle_propagate(prob, x_packed, nsteps, level=0, grid_sel=None):
    gl = solve.grid_list(prob)
    dt = propagate.step_size(prob, level)
    parts = split(prob, x_packed)
    sel = range(len(gl)) if grid_sel is None else grid_sel
    return [propagate.march(prob, gl[g][0], parts[g], nsteps, dt) for g in sel]


def oracle_initial(prob):
    gl = solve.grid_list(prob)
    return np.concatenate([grids.initial_value(prob, l) for (l, _, _) in gl])


def oracle_mgrit_history(prob, nit, grid_sel=None):
    """Per-iteration max over grids of max_m ||r_m|| / ||u0_g|| from the
    oracle's MGRIT (first `nit` iterations)."""
    from oracle import mgrit
    gl = solve.grid_list(prob)
    N, c, L = prob["nsteps"], prob["cf"], prob["mgrit_levels"]
    dt = propagate.step_size(prob, 0)
    sel = range(len(gl)) if grid_sel is None else grid_sel
    hist = np.zeros(nit)
    for g in sel:
        l = gl[g][0]
        u0 = grids.initial_value(prob, l)
        phis = [propagate.Propagator(prob, l, dt * c ** k) for k in range(L)]
        h = []
        mgrit.solve(phis, u0, N, c, 0.0, nit, prob.get("relax", "FCF"), history=h)
        hist = np.maximum(hist, np.array(h) / max(np.linalg.norm(u0), 1e-300))
    return hist


__all__ = ["rel_l2", "split", "oracle_apply", "oracle_abs_apply", "oracle_propagate",
           "oracle_initial", "oracle_mgrit_history", "combine", "index_set", "solve"]
