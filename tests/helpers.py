"""Shared helpers of the GPU parity tests: run the oracle and the HIP path
on the same seeded problem and compare."""
import os

import numpy as np

from oracle import combine, grids, index_set, operators, propagate, sde, solve

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def state_errors(prob, u, ref, floor=1e-6):
    """(whole-state relative L2, largest per-grid relative L2, largest
    element error over the state's max norm). A grid's error is taken
    relative to its own norm, or to `floor` times the largest grid norm when
    its solution is smaller than that (grids on which the initial modes
    vanish hold rounding noise only)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    pu, pr = split(prob, u), split(prob, ref)
    norms = [np.linalg.norm(r) for r in pr]
    scale = floor * max(max(norms), 1e-300)
    grid = max(np.linalg.norm(a - b) / max(n, scale) for a, b, n in zip(pu, pr, norms))
    elem = np.abs(u - ref).max() / max(np.abs(ref).max(), 1e-300)
    return rel_l2(u, ref), float(grid), float(elem)


def assert_state_close(prob, u, ref, tol, what=""):
    """The solve-level parity bar: whole state, every grid and every element
    within tol (see state_errors)."""
    glob, grid, elem = state_errors(prob, u, ref)
    print(f"  {what} rel L2 {glob:.3e}, worst grid {grid:.3e}, worst element {elem:.3e} "
          f"(bar {tol:.0e})", flush=True)
    assert glob <= tol and grid <= tol and elem <= tol, (glob, grid, elem, tol)


def _oracle_part(prob, sel):
    return sel, solve.component_states(prob, sel)


def oracle_states(prob, workers=None):
    """Every component state at T from the oracle; large workloads spread
    the grids over host processes (spawned, so the GPU context of the test
    process is not inherited)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    gl = solve.grid_list(prob)
    sizes = np.diff(solve.offsets(prob))
    work = int(sizes.sum()) * prob["nsteps"]
    if workers is None:
        try:
            ncpu = len(os.sched_getaffinity(0))
        except AttributeError:
            ncpu = os.cpu_count() or 1
        workers = max(1, min(16, ncpu)) if work > 5e7 else 1
    if workers == 1:
        return solve.component_states(prob)
    bins = [[] for _ in range(workers)]
    load = [0] * workers
    for g in sorted(range(len(gl)), key=lambda g: -sizes[g]):
        b = load.index(min(load))
        bins[b].append(g)
        load[b] += int(sizes[g])
    bins = [b for b in bins if b]
    states = [None] * len(gl)
    with cf.ProcessPoolExecutor(len(bins), mp_context=mp.get_context("spawn")) as ex:
        for sel, st in ex.map(_oracle_part, [prob] * len(bins), bins):
            for g, x in zip(sel, st):
                states[g] = x
    return states


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


def table3_figures():
    """Table 3 of Section 4.4.1: scheme -> maximum error at the origin."""
    rows = {}
    with open(os.path.join(GOLD, "table3_oscillator_origin.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                rows[k] = float(v)
    return rows


def origin_errors(series, coef, every, dt):
    """|u^(c)(0, t) - p(0, t)| at the sampled times of a stored origin series
    of the 2-D oscillator (the origin is a node of every component grid, so
    the combination there is the coefficient sum of the grid values)."""
    from workloads import make
    p = make("fp_osc2d")
    th, H = np.asarray(p["drift"]), np.diag(p["diffusion"])
    comb = np.asarray(coef) @ np.asarray(series)
    out = np.empty(comb.shape[0])
    for k in range(comb.shape[0]):
        m, C = sde.moments(th, H, p["mean0"], np.diag(p["var0"]), k * every * dt)
        out[k] = abs(comb[k] - sde.density(np.zeros((1, 2)), m, C)[0])
    return out


__all__ = ["rel_l2", "split", "state_errors", "assert_state_close", "oracle_states", "oracle_apply", "oracle_abs_apply", "oracle_propagate",
           "oracle_initial", "oracle_mgrit_history", "table3_figures",
           "origin_errors", "GOLD", "combine", "index_set", "solve"]
