"""Launch shapes, schedules and their autotuner (through the C ABI): every
admissible shape of a grid gives the oracle's solution to the usual bars,
both MGRIT schedules give the same bits, invalid settings are rejected, and
the autotuned plan keeps parity, also at the size and settings of the 3-D
heat measurement."""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2509_22156_amd import ctm  # noqa: E402
from workloads import make, metric_settings  # noqa: E402

from helpers import assert_state_close, rel_l2, solve  # noqa: E402

WAVES = (1, 2, 4, 8, 16)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small(name):
    return make(name, **{
        "heat3d": dict(n=6, nsteps=64, t1=0.05),
        "ou4d": dict(n=5, nsteps=64, t1=0.25),
        "cme5d": dict(d=3, n=4, hi=[16.0] * 3, nsteps=32, t1=0.5),
        "varcoef6d": dict(d=4, n=4, nsteps=64, t1=0.02, cf=4),
        "fp_lin4d": dict(n=5, nsteps=32),
    }[name])


def _settings(p, prec):
    p = dict(p)
    if prec == "fp64":
        p.update(prec="fp64", krylov_tol=1e-13, mgrit_tol=1e-13, mgrit_maxit=100)
    else:
        p.update(prec="mixed", refine_tol=1e-12, inner_tol=1e-5, mgrit_tol=1e-11,
                 krylov_tol=1e-13, mgrit_maxit=100)
    return p


def _move_to_other_k(plan):
    """Give every on-chip grid the other number of unknowns per lane, with
    the fewest waves the solver accepts; returns how many grids moved."""
    moved = 0
    for g in range(plan.G):
        w0, k0 = plan.grid_shape(g)
        if k0 == 0:
            continue
        k1 = 8 if k0 == 4 else 4
        for w in WAVES:
            try:
                plan.set_grid_shape(g, w, k1)
            except ctm.CtmError:
                continue
            assert plan.grid_shape(g) == (w, k1)
            moved += 1
            break
    return moved


@pytest.mark.parametrize("name", ["heat3d", "ou4d", "cme5d", "varcoef6d", "fp_lin4d"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_other_shapes_same_solution(name, prec):
    p = _settings(_small(name), prec)
    _say(f"other shapes {name} {prec}")
    plan = ctm.Plan(p)
    assert _move_to_other_k(plan) > 0
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    ref = solve.packed(solve.component_states(p))
    assert st["status_flags"] == 0
    assert_state_close(p, u, ref, (1e-11 if prec == "fp64" else 1e-8))


def test_set_grid_shape_rejects_invalid():
    p = _settings(_small("heat3d"), "fp64")
    plan = ctm.Plan(p)
    for bad in [(3, 4), (4, 6), (0, 4), (32, 8)]:
        with pytest.raises(ctm.CtmError, match="no such launch shape"):
            plan.set_grid_shape(0, *bad)
    with pytest.raises(ctm.CtmError, match="out of range"):
        plan.set_grid_shape(plan.G, 1, 4)
    # at level 8 some grids need more than one wave's lanes at K = 4
    big = ctm.Plan(_settings(make("heat3d", n=8, nsteps=64, t1=0.05), "fp64"))
    rejected = 0
    for g in range(big.G):
        w, k = big.grid_shape(g)
        if w > 1 and k == 4:
            with pytest.raises(ctm.CtmError, match="cannot hold"):
                big.set_grid_shape(g, 1, 4)
            assert big.grid_shape(g) == (w, k)
            rejected += 1
    assert rejected > 0


@pytest.mark.parametrize("name", ["heat3d", "ou4d"])
def test_autotune_keeps_parity(name):
    p = _settings(_small(name), "mixed")
    _say(f"autotune {name}")
    plan = ctm.Plan(p)
    rep = plan.autotune(trial_iterations=2, repeats=1)
    assert rep["classes"] >= 1
    # the default shapes, one trial per class, one for the other schedule
    assert rep["trials"] == 2 + rep["classes"]
    assert rep["schedule"] in (ctm.SCHED_AUTO, ctm.SCHED_JOINED, ctm.SCHED_PER_CLASS)
    assert 0 < rep["ms_tuned"] <= rep["ms_default"]
    assert 0 <= rep["changed"] <= rep["classes"]
    for g in range(plan.G):
        w, k = plan.grid_shape(g)
        assert w in WAVES and k in (4, 8)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    ref = solve.packed(solve.component_states(p))
    assert st["status_flags"] == 0
    assert_state_close(p, u, ref, 1e-8)


def test_autotune_full_heat3d_measurement_settings():
    # the configuration the benchmark times: full size, mixed, tuned shapes
    p = make("heat3d", prec="mixed")
    p.update(metric_settings("mixed"))
    _say("autotune heat3d full size")
    plan = ctm.Plan(p)
    rep = plan.autotune(trial_iterations=3, repeats=1)
    _say(f"report {rep}")
    assert rep["trials"] == 2 + rep["classes"]
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    assert st["status_flags"] == 0
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, u, ref, 1e-8)


@pytest.mark.parametrize("name,prec,levels", [("heat3d", "mixed", 2), ("ou4d", "fp64", 3),
                                              ("ou4d", "mixed", 3), ("varcoef6d", "mixed", 3)])
def test_schedules_give_identical_results(name, prec, levels):
    # joined phases and per-class lanes run the same kernels on the same
    # data: the states agree bit for bit, and both meet the oracle
    p = _settings(_small(name), prec)
    p["mgrit_levels"] = levels
    _say(f"schedules {name} {prec} levels={levels}")
    out, its = {}, {}
    for sched in (ctm.SCHED_JOINED, ctm.SCHED_PER_CLASS):
        plan = ctm.Plan(p)
        plan.set_schedule(sched)
        out[sched] = plan.solve().cpu().numpy()
        st = plan.stats()
        assert st["status_flags"] == 0
        its[sched] = st["mgrit_iterations"]
    assert its[ctm.SCHED_JOINED] == its[ctm.SCHED_PER_CLASS]
    assert (out[ctm.SCHED_JOINED] == out[ctm.SCHED_PER_CLASS]).all()
    ref = solve.packed(solve.component_states(p))
    assert_state_close(p, out[ctm.SCHED_PER_CLASS], ref, 1e-11 if prec == "fp64" else 1e-8)


def test_set_schedule_rejects_unknown():
    plan = ctm.Plan(_settings(_small("heat3d"), "fp64"))
    for bad in (-1, 3):
        with pytest.raises(ctm.CtmError, match="unknown schedule"):
            plan.set_schedule(bad)
