"""GPU parity of the streaming path: component grids beyond the on-chip
solver (lines longer than 512 unknowns, or more than 8,192 unknowns) are
solved with their Krylov vectors in HBM - by the wide solver (many
work-groups per system, the default) or by the one-work-group-per-system
streaming kernel - alongside the on-chip grids of the same plan."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2509_22156_amd import ctm  # noqa: E402
from workloads import make, random_vectors  # noqa: E402

from helpers import (assert_state_close, combine, oracle_abs_apply, oracle_apply, oracle_mgrit_history,  # noqa: E402
                     oracle_propagate, rel_l2, solve, split)


ALL = 1 << 20  # set_wide: every streaming launch on the wide solver


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _heat2d_big(**kw):
    # level 10: the grids (10, 1) and (1, 10) have lines of 1,023 unknowns
    p = make("heat2d", n=10, nsteps=32, t1=0.05)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100, cf=4)
    p.update(kw)
    return p


def test_streaming_classes_present():
    plan = ctm.Plan(_heat2d_big())
    plan.solve()
    shapes = plan.stats()["shapes"]
    assert any(s["K"] == 0 for s in shapes) and any(s["K"] > 0 for s in shapes), shapes


def test_set_wide_rejects_a_negative_count():
    plan = ctm.Plan(_heat2d_big())
    with pytest.raises(ctm.CtmError):
        plan.set_wide(-1)
    plan.set_wide(0)
    plan.set_wide(1 << 30)  # capped


def test_streaming_grids_keep_their_shape():
    plan = ctm.Plan(_heat2d_big())
    stream = [g for g in range(plan.G) if plan.grid_shape(g) == (16, 0)]
    assert stream
    with pytest.raises(ctm.CtmError, match="streaming"):
        plan.set_grid_shape(stream[0], 16, 8)
    rep = plan.autotune(trial_iterations=1, repeats=1)
    assert all(plan.grid_shape(g) == (16, 0) for g in stream), rep


def test_streaming_apply():
    p = _heat2d_big()
    plan = ctm.Plan(p)
    x = random_vectors(plan.slen, 1, seed=31)[0]
    y = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle_apply(p, x)
    bound = 16 * np.finfo(np.float64).eps * oracle_abs_apply(p, x)
    assert (np.abs(y - ref) <= bound + 1e-300).all()


@pytest.mark.parametrize("kw", [dict(mgrit_levels=1), dict(), dict(relax="F"),
                                dict(krylov="bicgstab"), dict(nrecomb=2)])
def test_streaming_solve_fp64(kw):
    p = _heat2d_big(**kw)
    _say(f"streaming heat2d n=10 {kw}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("relax", ["FCF", "F"])
def test_streaming_mgrit_residual_history(relax):
    # the first iterations' C-point residuals pin relaxation, restriction,
    # coarse solve and correction on the streaming grids too
    p = _heat2d_big(mgrit_maxit=3, mgrit_tol=1e-300, relax=relax)
    _say(f"streaming mgrit history {relax}")
    plan = ctm.Plan(p)
    u, st_code = plan.solve(check=False)
    assert st_code == ctm.ERR_NOCONV
    hist = plan.stats()["mgrit_residual"]
    ref = oracle_mgrit_history(p, 3)
    assert len(hist) == 3
    for a, b in zip(hist, ref):
        assert abs(a - b) <= 1e-7 * b + 1e-13, (hist, ref)


def test_streaming_solve_mixed():
    p = _heat2d_big(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
                    coarse_tol=1e-3)
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("name,kw", [("ou4d", dict(d=2, n=10, nsteps=16, t1=0.1)),
                                     ("cme5d", dict(d=2, n=10, hi=[1024.0] * 2, nsteps=16, t1=0.1)),
                                     ("varcoef6d", dict(d=2, n=10, nsteps=16, t1=0.01, cf=4)),
                                     ("fp_osc2d", dict(n=12, L0=3, nsteps=16, t1=0.08))])
def test_streaming_other_operators(name, kw):
    p = make(name, **kw)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100)
    _say(f"streaming {name} {kw}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    assert any(s["K"] == 0 for s in plan.stats()["shapes"])
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("name,kw", [("varcoef6d", dict(d=2, n=10, nsteps=16, t1=0.01, cf=4)),
                                     ("fp_osc2d", dict(n=12, L0=3, nsteps=16, t1=0.08)),
                                     ("ou4d", dict(d=2, n=10, nsteps=16, t1=0.1)),
                                     ("cme5d", dict(d=2, n=10, hi=[1024.0] * 2, nsteps=16,
                                                    t1=0.1))])
def test_streaming_mixed_other_operators(name, kw):
    # mixed plans: the on-chip grids by FP32 correction solves with FP64
    # refinement (their coarse MGRIT levels in FP64), the streaming grids on
    # the wide solver in FP64 with its line factors stored in FP32 (CG for
    # the variable coefficient, BiCGStab for the drift, OU and CME
    # operators); the mixed bar against the oracle
    p = make(name, **kw)
    p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
             mgrit_maxit=100, coarse_tol=1e-3)
    _say(f"streaming mixed {name} {kw}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    assert any(s["K"] == 0 for s in plan.stats()["shapes"])
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("name,kw", [("heat2d", dict(nrecomb=2)),
                                     ("heat2d", dict(mgrit_levels=3, cf=2)),
                                     ("varcoef6d", dict(nrecomb=2)),
                                     ("varcoef6d", dict(mgrit_levels=3, cf=2))])
def test_streaming_mixed_recombination_and_levels(name, kw):
    # mixed plans with streaming grids, with two recombination blocks
    # (s = 2) or three MGRIT levels (FP64 coarse launches of every class)
    if name == "heat2d":
        p = _heat2d_big(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
                        coarse_tol=1e-3)
    else:
        # (three MGRIT levels by default: 32 steps keep each of two
        # recombination blocks divisible by cf^2)
        p = make(name, d=2, n=10, nsteps=32, t1=0.01, cf=4)
        p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
                 mgrit_maxit=100, coarse_tol=1e-3)
    p.update(kw)
    _say(f"streaming mixed {name} {kw}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


def test_streaming_mixed_plan_per_grid_propagation():
    # the per-grid propagation of a mixed plan runs every class in FP64
    # (the layout its size classes must also fit), streaming grids included
    p = make("fp_osc2d", n=12, L0=3, nsteps=16, t1=0.08)
    p.update(prec="mixed", krylov_tol=1e-13, refine_tol=1e-12, inner_tol=1e-5)
    plan = ctm.Plan(p)
    x = random_vectors(plan.slen, 1, seed=37)[0]
    y = plan.propagate(torch.from_numpy(x).cuda(), 2, per_grid=True).cpu().numpy()
    ref = np.concatenate(oracle_propagate(p, x, 2))
    parts, rparts = split(p, y), split(p, ref)
    for a, b in zip(parts, rparts):
        assert rel_l2(a, b) <= 1e-11


@pytest.mark.parametrize("kw", [dict(mgrit_levels=1), dict(), dict(krylov="bicgstab"),
                                dict(relax="F", cf=8), dict(krylov="bicgstab", mgrit_levels=1)])
def test_streaming_wide_against_narrow(kw):
    # the same solve with every streaming launch on the wide solver (many
    # work-groups per task), and with none (one work-group per task): both
    # meet the oracle, and agree with each other to the Krylov tolerance
    p = _heat2d_big(**kw)
    out = {}
    for wide in (0, ALL):
        _say(f"streaming wide={wide} {kw}")
        plan = ctm.Plan(p)
        plan.set_wide(wide)
        out[wide] = plan.solve().cpu().numpy()
        st = plan.stats()
        assert st["status_flags"] == 0
        assert st["krylov_iterations"] > 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, out[0], ref, 1e-11)
    assert_state_close(p, out[ALL], ref, 1e-11)
    assert_state_close(p, out[ALL], out[0], 1e-11)


def test_streaming_wide_drift_oscillator():
    # the full-drift operator (BiCGStab) with every streaming launch wide
    p = make("fp_osc2d", n=12, L0=3, nsteps=16, t1=0.08)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100)
    _say("streaming wide fp_osc2d")
    plan = ctm.Plan(p)
    plan.set_wide(ALL)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


def test_streaming_wide_noconv_flag():
    # a Krylov cap the tolerance cannot meet: the wide solver stops at the
    # cap and reports non-convergence, like the one-work-group kernel
    p = _heat2d_big(mgrit_levels=1, krylov_maxit=2, krylov_tol=1e-14)
    for wide in (0, ALL):
        plan = ctm.Plan(p)
        plan.set_wide(wide)
        _, code = plan.solve(check=False)
        assert code == ctm.ERR_NOCONV, wide
        assert plan.stats()["krylov_max"] == 2, wide


@pytest.mark.parametrize("kw", [dict(mgrit_levels=1), dict(), dict(krylov="bicgstab")])
def test_streaming_three_dimensional(kw):
    # d = 3 (the dimension bound 4 of both streaming solvers): at level 10
    # the grids (10,1,1), (1,10,1), (1,1,10) have lines of 1,023 unknowns
    # and run on the streaming solvers, the other 133 on chip
    p = make("heat3d", n=10, nsteps=16, t1=0.01)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100, cf=4)
    p.update(kw)
    ref = solve.packed(solve.component_states(p))
    for wide in (0, ALL):
        _say(f"streaming heat3d n=10 wide={wide} {kw}")
        plan = ctm.Plan(p)
        plan.set_wide(wide)
        u = plan.solve().cpu().numpy()
        st = plan.stats()
        assert st["status_flags"] == 0
        assert any(s["K"] == 0 for s in st["shapes"])
        assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("krylov", ["cg", "bicgstab"])
def test_streaming_wide_many_tasks(krylov):
    # 128 intervals x 2 streaming grids: relaxation launches of 256 tasks,
    # where the wide solver stages the lines of the grid whose stiff axis is
    # its fastest axis through LDS; against the oracle and the one-work-group
    # kernel
    p = _heat2d_big(nsteps=256, cf=2, krylov=krylov)
    ref = solve.packed(solve.component_states(p))
    out = {}
    for wide in (0, ALL):
        _say(f"streaming many tasks wide={wide} {krylov}")
        plan = ctm.Plan(p)
        plan.set_wide(wide)
        out[wide] = plan.solve().cpu().numpy()
        assert plan.stats()["status_flags"] == 0
        assert_state_close(p, out[wide], ref, 1e-11)
    assert_state_close(p, out[ALL], out[0], 1e-11)


@pytest.mark.parametrize("nsteps", [20, 28, 36])
@pytest.mark.parametrize("krylov", ["cg", "bicgstab"])
def test_streaming_wide_task_groups(nsteps, krylov):
    # 2 streaming grids x nsteps / 4 intervals: relaxation launches of 10,
    # 14 and 18 tasks, i.e. full groups of eight tasks (each task's
    # work-groups on one XCD) together with a last group of 2, 6 and 2 in
    # plain order; against the oracle
    p = _heat2d_big(nsteps=nsteps, cf=4, krylov=krylov)
    _say(f"streaming task groups nsteps={nsteps} {krylov}")
    plan = ctm.Plan(p)
    plan.set_wide(ALL)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("tight", [False, True])
def test_streaming_paper_size_oscillator(tight):
    # the benchmark's streaming workload at full size (Section 4.4, L = 14,
    # L0 = 6: 7 grids, 177,415 unknowns per level, 256 steps, every grid on
    # the wide solver): with the measurement tolerances (MGRIT 1e-9 on the
    # C-point residual, the final state's error then ~1e-8) and with tight
    # ones, against the oracle
    p = make("fp_osc2d", n=14, L0=6, prec="fp64")
    if tight:
        p.update(krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100, krylov_maxit=20000)
    else:
        p.update(krylov_tol=1e-10, mgrit_tol=1e-9, mgrit_maxit=64, krylov_maxit=20000,
                 coarse_tol=1e-3)
    _say(f"paper-size oscillator tight={tight}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, (1e-10 if tight else 5e-8))


@pytest.mark.parametrize("name,kw", [("varcoef6d", dict(d=2, n=10, nsteps=256, t1=0.01, cf=2)),
                                     ("cme5d", dict(d=2, n=10, hi=[1024.0] * 2, nsteps=256,
                                                    t1=0.1, cf=2))])
def test_streaming_many_tasks_with_tables(name, kw):
    # relaxation launches of more than 64 tasks (staged line sweeps) for the
    # operators whose coefficient tables the kernels keep in LDS beside the
    # line tile
    p = make(name, **kw)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100)
    _say(f"streaming many tasks {name}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    assert any(s["K"] == 0 for s in plan.stats()["shapes"])
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


def test_drift_beyond_the_solver_reports_noconv():
    # the oscillator's step is dt = 0.005 (Section 4.4.1); at 16 times that
    # step (coarse step 0.16) the central fluxes of the rotating drift give
    # the mid-size grids a spectrum far off the real axis, where BiCGStab with
    # the line preconditioner stagnates: the solve must end with that
    # reported (no convergence, or a breakdown once MGRIT has diverged)
    p = make("fp_osc2d", n=12, L0=3, nsteps=16)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=4, krylov_maxit=200)
    _say("drift at 16x the paper's step")
    plan = ctm.Plan(p)
    _, st = plan.solve(check=False)
    flags = plan.stats()["status_flags"]
    assert st in (ctm.ERR_NOCONV, ctm.ERR_BREAKDOWN)
    assert flags & (1 << ctm.ERR_NOCONV)


def test_lines_cut_into_segments_mixed():
    # the level-12 case in a mixed plan: on-chip grids by FP32 corrections
    # with FP64 refinement, the segmented streaming grids in FP64 on the
    # wide solver (FP32 line factors)
    p = make("heat2d", n=12, nsteps=8, t1=1e-4)
    p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
             mgrit_maxit=100, cf=2, krylov_maxit=20000, coarse_tol=1e-3)
    _say("segmented lines mixed n=12")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("n,wide", [(12, ALL), (12, 0), (13, ALL), (13, 0)])
def test_lines_cut_into_segments(n, wide):
    # levels 12 and 13: the grids (n, 1), (n - 1, 1), ... have lines of up to
    # 4,095 and 8,191 unknowns, longer than one wave's 1,024-unknown segment
    # of the line preconditioner (two to eight segments, the last shorter or
    # full); the
    # operator couples across the segments, the preconditioner does not, so
    # the solution matches the oracle's direct solves as for any other grid,
    # on the wide solver and on the one-work-group-per-system kernel
    # (dt / h^2 about 50 and 200 on the finest axis: a condition number low
    # enough for FP64 CG to reach the tolerances; at dt / h^2 ~ 2e4 the gap
    # between the recursive and the true residual, eps times the condition
    # number, keeps the MGRIT residual above 1e-13)
    p = make("heat2d", n=n, nsteps=8, t1=1e-4)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-12, mgrit_maxit=100, cf=2,
             krylov_maxit=20000)
    gl = solve.grid_list(p)
    assert max(2 ** max(l) - 1 for (l, _, _) in gl) > 1024
    _say(f"segmented lines n={n} wide={wide}")
    plan = ctm.Plan(p)
    plan.set_wide(wide)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    _say(f"  mgrit it={st['mgrit_iterations']} krylov={st['krylov_iterations']}")
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)
