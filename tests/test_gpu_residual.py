"""MGRIT in space-time residual mode (the optimized oscillator run of
Section 4.4): fixed-count inexact implicit steps, exact space-time
residuals and the residual form of the coarse equation. The fixed point is
the time-sequential solution, so the converged result is compared with the
oracle's element by element; at the paper's own settings (c = 12,
F-relaxation, residual tolerance 1e-4, two Krylov iterations per step) the
result is held to the accuracy such a tolerance gives."""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2509_22156_amd import ctm  # noqa: E402
from workloads import make  # noqa: E402

from helpers import assert_state_close, rel_l2, solve  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small(name):
    return make(name, **{
        "heat3d": dict(n=6, nsteps=64, t1=0.05),
        "ou4d": dict(n=5, nsteps=64, t1=0.25),  # three levels
        "fp_osc2d": dict(n=9, L0=4, nsteps=32),
        "fp_lin4d": dict(n=5, nsteps=32, prec="fp64"),
    }[name])


RES = dict(prec="fp64", residual_mode=1, krylov_maxit=2, mgrit_tol=1e-12, mgrit_maxit=400)


@pytest.mark.parametrize("name", ["heat3d", "ou4d", "fp_osc2d", "fp_lin4d"])
@pytest.mark.parametrize("relax", ["FCF", "F"])
def test_residual_mode_reaches_sequential_solution(name, relax):
    p = _small(name)
    p.update(RES, relax=relax)
    _say(f"residual mode {name} {relax}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    assert st["mgrit_residual"][-1] <= p["mgrit_tol"]
    # two Krylov iterations per step: the work per solve is bounded
    assert st["krylov_max"] <= p["krylov_maxit"]
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("name", ["heat3d", "ou4d", "fp_lin4d"])
def test_residual_mode_mixed_precision(name):
    # one FP32 correction solve of two iterations per step on the FP64
    # residual; the space-time residual is FP64, so the fixed point is the
    # same
    p = _small(name)
    p.update(RES, prec="mixed", mgrit_tol=1e-11)
    _say(f"residual mode mixed {name}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


def test_residual_mode_paper_settings_oscillator():
    # Section 4.4, optimized run: T = 1, c = 12, F-relaxation, two temporal
    # levels, residual tolerance 1e-4, two iterations of the spatial solver
    # per step (N = 3204 = 12 * 267 steps: dt = 1/3204 for the paper's
    # 1/3200, which is not a multiple of 12)
    p = make("fp_osc2d", t1=1.0, nsteps=3204)
    p.update(cf=12, relax="F", prec="fp64", krylov_maxit=2, residual_mode=1, mgrit_tol=1e-4,
             mgrit_maxit=100)
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    _say(f"  iterations {st['mgrit_iterations']} residuals {st['mgrit_residual']}")
    assert st["status_flags"] == 0 and st["mgrit_residual"][-1] <= 1e-4
    ref = solve.packed(solve.component_states(p))
    err = rel_l2(u, ref)
    _say(f"  rel. L2 against the sequential solution {err:.2e}")
    # the tolerance bounds every step's space-time residual at 1e-4 of
    # ||u0||; with a non-expansive propagator the state error is at most the
    # sum of the residuals over the steps (a useless 0.3 here). The bar is
    # empirical: 1e-3, against ~5e-6 measured on MI355X.
    assert err <= 1e-3


@pytest.mark.parametrize("relax", ["FCF", "F"])
def test_residual_mode_streaming_grids_mixed(relax):
    # mixed plan: the on-chip grids by one FP32 correction solve per step,
    # the streaming grids in FP64 (wide solver); FP64 space-time residual
    p = make("heat2d", n=10, nsteps=32, t1=0.05)
    p.update(RES, relax=relax, cf=4, prec="mixed", mgrit_tol=1e-11)
    _say(f"residual mode mixed with streaming grids {relax}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert any(s["K"] == 0 for s in st["shapes"])
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("relax", ["FCF", "F"])
def test_residual_mode_streaming_grids(relax):
    # level 10: the grids (10, 1) and (1, 10) run on the streaming kernel
    p = make("heat2d", n=10, nsteps=32, t1=0.05)
    p.update(RES, relax=relax, cf=4)
    _say(f"residual mode with streaming grids {relax}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert any(s["K"] == 0 for s in st["shapes"])
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("tol,bar", [(1e-10, 1e-9), (1e-4, 1e-3)])
def test_residual_mode_paper_level_oscillator(tol, bar):
    # the paper's own levels (L = 14, L0 = 6, every grid on the streaming
    # path) with the optimized run's settings, on a shorter interval (288
    # steps of 1/3204) so that the oracle finishes in seconds
    p = make("fp_osc2d", n=14, L0=6, t1=288 / 3204, nsteps=288)
    p.update(cf=12, relax="F", prec="fp64", krylov_maxit=2, residual_mode=1, mgrit_tol=tol,
             mgrit_maxit=200)
    _say(f"residual mode paper-level oscillator tol={tol}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    _say(f"  iterations {st['mgrit_iterations']}")
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    err = rel_l2(u, ref)
    _say(f"  rel. L2 against the sequential solution {err:.2e}")
    assert err <= bar
