"""GPU parity of the two-level overlapping Schwarz preconditioner (Section
2.1.2; balanced with CG, additive with BiCGStab as in Section 4.1), through
the C ABI: the preconditioner itself against the oracle's dense matrices,
grid by grid and element by element; the preconditioned solves against the
oracle's direct solves; the preconditioned Krylov iteration counts against
the oracle's preconditioned solvers; and the rejections."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2509_22156_amd import ctm  # noqa: E402
from workloads import make, random_vectors  # noqa: E402

from helpers import assert_state_close, oracle_states, solve, split  # noqa: E402
from oracle import krylov, operators, propagate, schwarz  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# small problems of every operator class (CG: heat, varcoef; BiCGStab: ou,
# cme, drift), on several subdomain sizes 2^S
CASES = {
    "heat2d": dict(n=6, nsteps=16, t1=0.05, cf=4),
    "heat3d": dict(n=5, nsteps=16, t1=0.02, cf=4),
    "varcoef6d": dict(d=3, n=5, nsteps=16, t1=0.02, cf=4),
    "ou4d": dict(d=2, n=6, nsteps=16, t1=0.2, cf=4),
    "cme5d": dict(d=2, n=5, hi=[32.0] * 2, nsteps=16, t1=0.5, cf=4),
    "fp_osc2d": dict(n=8, L0=4, nsteps=16, t1=0.08, cf=2),
    "fp_lin4d": dict(n=5, nsteps=16, t1=0.064, cf=2),
}


def _problem(name, S, prec="fp64", **kw):
    p = make(name, **CASES[name])
    p.update(precond="schwarz", schwarz_s=S, prec=prec, krylov_tol=1e-13, mgrit_tol=1e-13,
             mgrit_maxit=100, krylov_maxit=5000)
    p.update(kw)
    return p


@pytest.mark.parametrize("name,S", [("heat2d", 3), ("heat2d", 5), ("heat3d", 4), ("varcoef6d", 4),
                                    ("ou4d", 4), ("cme5d", 3), ("fp_osc2d", 5),
                                    ("fp_lin4d", 4)])
def test_preconditioner_matches_oracle(name, S):
    p = _problem(name, S)
    _say(f"schwarz apply {name} S={S}")
    plan = ctm.Plan(p)
    gl = solve.grid_list(p)
    x = random_vectors(plan.slen, 1, seed=31)[0]
    xs = split(p, x)
    for level in (0, 1):
        y = plan.precond_apply(torch.from_numpy(x).cuda(), level=level).cpu().numpy()
        dt = propagate.step_size(p, level)
        for (l, _, _), xg, yg in zip(gl, xs, split(p, y)):
            C = schwarz.preconditioner(p, l, dt, S)
            ref = C @ xg
            err = np.abs(yg - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err <= 1e-11, (l, level, err)


@pytest.mark.parametrize("name,prec", [("heat3d", "fp64"), ("varcoef6d", "fp64"),
                                       ("ou4d", "fp64"), ("fp_lin4d", "fp64"),
                                       ("heat3d", "mixed"), ("cme5d", "fp64")])
def test_schwarz_solves_match_oracle(name, prec):
    p = _problem(name, 4, prec=prec)
    _say(f"schwarz solve {name} {prec}")
    plan = ctm.Plan(p)
    u = plan.solve().cpu().numpy()
    st = plan.stats()
    _say(f"  mgrit it={st['mgrit_iterations']} krylov={st['krylov_iterations']}")
    assert st["status_flags"] == 0
    assert all(c["K"] == 0 for c in st["shapes"])  # every grid on the streaming solver
    ref = solve.packed(oracle_states(p))
    assert_state_close(p, u, ref, 1e-11)


@pytest.mark.parametrize("name", ["heat3d", "varcoef6d", "ou4d", "fp_lin4d"])
def test_schwarz_iterations_match_oracle(name):
    # one implicit step from the initial value on every grid (x0 = b, the
    # streaming solver's start): the preconditioned CG / BiCGStab iteration
    # counts, summed over the grids, agree with the oracle's preconditioned
    # solvers on the same matrices and preconditioners
    p = _problem(name, 4, krylov_tol=1e-10)
    p["mgrit_levels"] = 1
    plan = ctm.Plan(p)
    u0 = plan.initial_state()
    plan.propagate(u0, 1)
    torch.cuda.synchronize()
    gpu_its = plan.stats()["krylov_iterations"]
    dt = propagate.step_size(p, 0)
    total = 0
    for (l, _, _), b in zip(solve.grid_list(p), split(p, u0.cpu().numpy())):
        A = operators.system_matrix(p, l, dt).toarray()
        C = schwarz.preconditioner(p, l, dt, 4)
        if operators.is_symmetric(p):
            _, it = krylov.pcg(A, b, C, x0=b.copy(), tol=1e-10)
        else:
            _, it = krylov.pbicgstab(A, b, C, x0=b.copy(), tol=1e-10)
        total += it
    _say(f"  {name}: GPU {gpu_its} oracle {total} Krylov iterations")
    assert abs(gpu_its - total) <= max(2, 0.05 * total)


def test_schwarz_rejections():
    for bad in (1, 7):
        with pytest.raises(ctm.CtmError, match="schwarz_s"):
            ctm.Plan(_problem("heat2d", bad))
    q = make("heat_mms", d=2, n=4, nsteps=8)
    q.update(precond="schwarz", schwarz_s=4)
    with pytest.raises(ctm.CtmError, match="manufactured"):
        ctm.Plan(q)
    # a dense coarse matrix of more than 1,024 blocks
    with pytest.raises(ctm.CtmError, match="coarse blocks"):
        ctm.Plan(_problem("heat2d", 5, n=15, L0=7, nsteps=4, t1=0.01))
    # the line-preconditioned plan has no Schwarz preconditioner to apply
    line = ctm.Plan(make("heat2d", **CASES["heat2d"]))
    x = torch.zeros(line.slen, dtype=torch.float64, device="cuda")
    with pytest.raises(ctm.CtmError, match="no Schwarz"):
        line.precond_apply(x)
    plan = ctm.Plan(_problem("heat2d", 4))
    with pytest.raises(ctm.CtmError, match="level out of range"):
        plan.precond_apply(torch.zeros(plan.slen, dtype=torch.float64, device="cuda"), level=2)
