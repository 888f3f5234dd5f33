"""GPU parity of the manufactured heat problem (Section 4.2): forcing
g_n = Phi dt f(t_n) in every level-0 implicit step, initial value u*(., t0),
against the CPU oracle on the same problem."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2509_22156_amd import ctm  # noqa: E402
from workloads import make  # noqa: E402

from helpers import assert_state_close, oracle_initial, oracle_propagate, rel_l2, solve  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fp64(**kw):
    p = make("heat_mms", **kw)
    p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100)
    return p


def test_manufactured_initial_state():
    p = _fp64(d=3, n=5)
    plan = ctm.Plan(p)
    got = plan.initial_state().cpu().numpy()
    ref = oracle_initial(p)
    assert np.abs(got - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max()) * 8


def test_manufactured_propagate():
    p = _fp64(d=3, n=5, nsteps=16, t1=0.5)
    plan = ctm.Plan(p)
    u0 = plan.initial_state()
    got = plan.propagate(u0, 6).cpu().numpy()
    ref = np.concatenate(oracle_propagate(p, u0.cpu().numpy(), 6))
    assert_state_close(p, got, ref, 1e-11)


@pytest.mark.parametrize("kw", [dict(d=2, n=6, mgrit_levels=1),
                                dict(d=2, n=6),
                                dict(d=3, n=5, cf=4),
                                dict(d=3, n=5, mgrit_levels=3, cf=2),
                                dict(d=4, n=4, nrecomb=2),
                                dict(d=3, n=5, relax="F")])
def test_manufactured_solve_fp64(kw):
    kw = dict(kw)
    base = {k: kw.pop(k) for k in ("d", "n") if k in kw}
    p = _fp64(nsteps=32, t1=0.5, **base)
    p.update(kw)
    _say(f"manufactured fp64 {base} {kw}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


def test_manufactured_solve_mixed():
    p = make("heat_mms", d=3, n=6, nsteps=32, t1=0.5)
    p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11, krylov_tol=1e-13,
             mgrit_maxit=100, coarse_tol=1e-3)
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    assert plan.stats()["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


def test_mgrit_iterations_independent_of_dimension_and_level():
    # Section 4.2 reports MGRIT iteration counts that do not grow with d,
    # the level L or the anisotropy of the grids (within a factor of 2)
    its = {}
    for d, n in [(2, 5), (2, 7), (3, 5), (3, 7), (4, 5), (5, 5)]:
        p = make("heat_mms", d=d, n=n, nsteps=32, t1=1.0)
        p.update(prec="fp64", krylov_tol=1e-10, mgrit_tol=1e-8, mgrit_maxit=64)
        plan = ctm.Plan(p)
        plan.solve()
        its[(d, n)] = plan.stats()["mgrit_iterations"]
    _say(f"MGRIT iterations {its}")
    assert max(its.values()) <= 2 * min(its.values()), its


def test_manufactured_on_streaming_grids_mixed():
    # the same in a mixed plan: the on-chip grids by FP32 corrections with
    # FP64 refinement, the streaming grids in FP64 on the wide solver, the
    # forcing added per point in both
    p = _fp64(d=2, n=12, nsteps=8, t1=2e-3)
    p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
             krylov_maxit=20000, cf=2)
    _say("manufactured on streaming grids, mixed")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    assert any(c["K"] == 0 for c in st["shapes"])
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("wide", [1 << 20, 0])
def test_manufactured_on_streaming_grids(wide):
    # 2-D level 12: the grids with lines of 2,047 unknowns run on the
    # streaming solvers (their line preconditioner cut into segments),
    # which add dt f(t_j) point by point; the wide solver and the
    # one-work-group-per-system kernel (dt / h^2 about 1e3 on the finest
    # axis, so that FP64 CG reaches the tolerances)
    p = _fp64(d=2, n=12, nsteps=8, t1=2e-3)
    p.update(mgrit_tol=1e-12, krylov_maxit=20000, cf=2)
    _say(f"manufactured on streaming grids, wide={wide}")
    plan = ctm.Plan(p)
    plan.set_wide(wide)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    assert any(c["K"] == 0 for c in st["shapes"])  # a streaming class
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)
