"""Seeded synthetic problem definitions for the five benchmark workloads.

This module only draws random parameters and tabulates the initial data on
the finest one-dimensional node set; it holds none of the method's
arithmetic (no grids, no operators, no time stepping, no combination).
Both the CPU oracle and the GPU path consume the dictionaries it returns.

A problem dictionary has these keys:

  d, n, L0          dimension, combination level n (the paper's L) and
                    minimal level L0 (Section 2.1.1, eq. for u_L^(c))
  lo, hi            box Omega = prod [lo_i, hi_i]
  op                "heat" | "varcoef" | "ou" | "cme"
  amp               var-coef amplitude: a(x) = 1 + amp * prod sin(2 pi x_k)
  theta, sigma      OU drift rates (diagonal) and noise: dX = -theta X dt + sigma dW
  k, gamma          immigration and death rates per species (cme)
  t0, t1, nsteps    time interval and number of backward-Euler steps N
  nrecomb           number of recombination blocks s (Section 2.2.1)
  mgrit_levels, cf  MGRIT levels and coarsening factor c (Section 2.3.1)
  mgrit_tol, mgrit_maxit
  krylov            "cg" | "bicgstab"; krylov_tol, krylov_maxit
  prec              "fp64" | "mixed"; refine_tol, inner_tol, refine_maxit
  ic_w, ic_f        initial value u0(x) = sum_r ic_w[r] prod_i ic_f[r, i, J_i],
                    with ic_f[r, i, J] the r-th factor on axis i sampled at the
                    finest 1-D node x = lo_i + J (hi_i - lo_i) / 2^n, J = 0..2^n
"""
from __future__ import annotations

import math

import numpy as np

NAMES = ("heat2d", "heat3d", "ou4d", "cme5d", "varcoef6d")


def _finest_nodes(lo: float, hi: float, n: int) -> np.ndarray:
    return lo + (hi - lo) * np.arange(2 ** n + 1, dtype=np.float64) / 2 ** n


def _base(d, n, lo, hi, op, t1, nsteps, levels, cf, krylov, prec):
    return dict(
        d=d, n=n, L0=1, lo=[float(lo)] * d, hi=[float(hi)] * d, op=op,
        amp=0.0, theta=[0.0] * d, sigma=0.0, k=[0.0] * d, gamma=[0.0] * d,
        t0=0.0, t1=float(t1), nsteps=int(nsteps), nrecomb=1,
        mgrit_levels=int(levels), cf=int(cf), mgrit_tol=1e-13, mgrit_maxit=64,
        krylov=krylov, krylov_tol=1e-13, krylov_maxit=20000,
        prec=prec, refine_tol=1e-13, inner_tol=1e-5, refine_maxit=12,
    )


def _sin_product(prob, wavenumbers, weights):
    d, n = prob["d"], prob["n"]
    f = np.empty((len(weights), d, 2 ** n + 1))
    for r, kv in enumerate(wavenumbers):
        for i in range(d):
            x = _finest_nodes(prob["lo"][i], prob["hi"][i], n)
            f[r, i] = np.sin(math.pi * kv[i] * x)
    prob["ic_w"] = np.asarray(weights, dtype=np.float64)
    prob["ic_f"] = f
    return prob


def heat2d(seed: int = 0, prec: str = "fp64") -> dict:
    """Heat equation, d=2, level 6, u0 = prod sin(pi x_i), 64 steps on [0, 0.1],
    two-level MGRIT with c=4, CG."""
    p = _base(2, 6, 0.0, 1.0, "heat", 0.1, 64, 2, 4, "cg", prec)
    return _sin_product(p, [[1, 1]], [1.0])


def heat3d(seed: int = 0, prec: str = "mixed") -> dict:
    """Heat equation, d=3, level 9, u0 = sum of 3 sin-product modes with
    integer wavenumbers in 1..4 and N(0,1) amplitudes; 256 steps on [0, 0.05];
    two-level MGRIT with c=8; CG."""
    rng = np.random.default_rng(seed)
    kv = rng.integers(1, 5, size=(3, 3))
    amp = rng.standard_normal(3)
    p = _base(3, 9, 0.0, 1.0, "heat", 0.05, 256, 2, 8, "cg", prec)
    p["modes"] = kv.tolist()
    return _sin_product(p, kv.tolist(), amp.tolist())


def ou4d(seed: int = 0, prec: str = "mixed") -> dict:
    """Fokker-Planck equation of a 4-D Ornstein-Uhlenbeck process
    dX = -theta X dt + sigma dW, theta_i ~ U[0.5, 2], sigma = 1, on [-6, 6]^4;
    Gaussian initial density N(mu0, 0.25 I), mu0 ~ U[-1, 1]^4; level 8;
    512 steps on [0, 1]; three-level MGRIT with c=4; BiCGStab."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.5, 2.0, size=4)
    mu0 = rng.uniform(-1.0, 1.0, size=4)
    p = _base(4, 8, -6.0, 6.0, "ou", 1.0, 512, 3, 4, "bicgstab", prec)
    p["theta"] = theta.tolist()
    p["sigma"] = 1.0
    p["mu0"] = mu0.tolist()
    p["var0"] = 0.25
    f = np.empty((1, 4, 2 ** 8 + 1))
    for i in range(4):
        x = _finest_nodes(-6.0, 6.0, 8)
        f[0, i] = np.exp(-(x - mu0[i]) ** 2 / (2 * 0.25)) / math.sqrt(2 * math.pi * 0.25)
    p["ic_w"] = np.ones(1)
    p["ic_f"] = f
    return p


def _gaussian_tables(p, mean, var):
    d, n = p["d"], p["n"]
    f = np.empty((1, d, 2 ** n + 1))
    for i in range(d):
        x = _finest_nodes(p["lo"][i], p["hi"][i], n)
        f[0, i] = np.exp(-(x - mean[i]) ** 2 / (2 * var[i])) / math.sqrt(2 * math.pi * var[i])
    p["ic_w"] = np.ones(1)
    p["ic_f"] = f
    return p


def fp_osc2d(seed: int = 0, prec: str = "fp64") -> dict:
    """Fokker-Planck equation of the 2-D linear oscillator of Section 4.4:
    theta = [[0, 1], [-w0^2, -2 xi w0]] with w0 = 1, xi = 0.05, sigma =
    (0, 1)^T, D = 0.1 (H = diag(0, 0.2)); N((5, 5), I/9) start on
    [-10, 10]^2; dt = 0.005 as in the paper, N = 256 steps; level 12 with
    L0 = 6 (the paper's initial level; three grids fit the on-chip solver);
    two-level MGRIT with c = 2, BiCGStab. Nothing is drawn."""
    p = _base(2, 12, -10.0, 10.0, "drift", 256 * 0.005, 256, 2, 2, "bicgstab", prec)
    p["L0"] = 6
    p["drift"] = [[0.0, 1.0], [-1.0, -0.1]]
    p["diffusion"] = [0.0, 0.2]
    p["mean0"], p["var0"] = [5.0, 5.0], [1.0 / 9.0] * 2
    return _gaussian_tables(p, p["mean0"], p["var0"])


def fp_lin4d(seed: int = 0, prec: str = "mixed") -> dict:
    """Fokker-Planck equation of the 4-D two-mass system of Section 4.4:
    k1 = k2 = k3 = 1, c1 = c2 = 0.4, excitation on both velocities with
    D1 = D2 = 0.2 (H = diag(0, 0.8, 0, 0.8)); N(0, 0.5 I) start on
    [-6, 6]^4; dt = 20/5000 as in the paper, N = 256 steps; level 8;
    two-level MGRIT with c = 2, BiCGStab. Nothing is drawn."""
    p = _base(4, 8, -6.0, 6.0, "drift", 256 * 0.004, 256, 2, 2, "bicgstab", prec)
    k1 = k2 = k3 = 1.0
    c1 = c2 = 0.4
    p["drift"] = [[0.0, 1.0, 0.0, 0.0], [-(k1 + k2), -c1, k2, 0.0],
                  [0.0, 0.0, 0.0, 1.0], [k2, 0.0, -(k2 + k3), -c2]]
    p["diffusion"] = [0.0, 0.8, 0.0, 0.8]
    p["mean0"], p["var0"] = [0.0] * 4, [0.5] * 4
    return _gaussian_tables(p, p["mean0"], p["var0"])


def cme5d(seed: int = 0, prec: str = "mixed") -> dict:
    """Master equation of 5 independent immigration-death species on the
    lattice 0..63 per species; k_i ~ U[5, 20], gamma_i ~ U[0.5, 1.5]; all
    mass at the origin initially; level 6; 256 steps on [0, 2]; two-level
    MGRIT with c=2; BiCGStab."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(5.0, 20.0, size=5)
    gamma = rng.uniform(0.5, 1.5, size=5)
    p = _base(5, 6, 0.0, 64.0, "cme", 2.0, 256, 2, 2, "bicgstab", prec)
    p["k"] = k.tolist()
    p["gamma"] = gamma.tolist()
    f = np.zeros((1, 5, 2 ** 6 + 1))
    f[0, :, 0] = 1.0
    p["ic_w"] = np.ones(1)
    p["ic_f"] = f
    return p


def varcoef6d(seed: int = 0, prec: str = "mixed") -> dict:
    """Variable-coefficient heat equation u_t = div(a grad u),
    a = 1 + 0.5 prod sin(2 pi x_i), d=6, level 8, u0 = prod sin(pi x_i);
    1024 steps on [0, 0.1]; three-level MGRIT with c=8; CG."""
    p = _base(6, 8, 0.0, 1.0, "varcoef", 0.1, 1024, 3, 8, "cg", prec)
    p["amp"] = 0.5
    return _sin_product(p, [[1] * 6], [1.0])


def heat_mms(seed: int = 0, prec: str = "fp64", d: int = 3, n: int = 6, nsteps: int = 64,
             t1: float = 1.0) -> dict:
    """Heat equation on [0,1]^d with the manufactured solution of Section 4.2
    (forcing and initial value derived from it; nothing is drawn, the seed
    is accepted for a uniform interface). Two-level MGRIT with c = 2 and
    FCF-relaxation, CG, as in the paper's solver setting (Section 4.1)."""
    p = _base(d, n, 0.0, 1.0, "heat", t1, nsteps, 2, 2, "cg", prec)
    p["manufactured"] = "heat"
    p["ic_w"] = [0.0]
    p["ic_f"] = np.zeros((1, d, 2 ** n + 1))
    return p


def make(name: str, seed: int = 0, **overrides) -> dict:
    """Problem dictionary of a named workload with optional field overrides.
    Overriding n or the box re-tabulates nothing: pass a fresh ic via
    overrides or use `retabulate`."""
    if name == "heat_mms":
        kw = {k: overrides.pop(k) for k in ("prec", "d", "n", "nsteps", "t1") if k in overrides}
        p = heat_mms(seed, **kw)
        p.update(overrides)
        return p
    fn = {"heat2d": heat2d, "heat3d": heat3d, "ou4d": ou4d, "cme5d": cme5d,
          "varcoef6d": varcoef6d, "fp_osc2d": fp_osc2d, "fp_lin4d": fp_lin4d}[name]
    kw = {}
    if "prec" in overrides:
        kw["prec"] = overrides["prec"]
    p = fn(seed, **kw)
    retab = any(k in overrides for k in ("n", "d", "lo", "hi"))
    p.update(overrides)
    if retab:
        p = retabulate(p, seed)
    return p


def retabulate(p: dict, seed: int = 0) -> dict:
    """Re-tabulate the initial factors after d, n or the box changed,
    keeping the workload's initial-value family."""
    d, n = p["d"], p["n"]
    for key in ("lo", "hi", "theta", "k", "gamma"):
        v = list(p[key])
        p[key] = (v + [v[-1]] * d)[:d]
    if p["op"] in ("heat", "varcoef"):
        modes = p.get("modes")
        if modes is None:
            return _sin_product(p, [[1] * d], [1.0])
        kv = [(list(m) + [1] * d)[:d] for m in modes]
        return _sin_product(p, kv, list(p["ic_w"]))
    if p["op"] == "drift":
        return _gaussian_tables(p, p["mean0"], p["var0"])
    if p["op"] == "ou":
        mu0 = (list(p.get("mu0", [0.0])) + [0.0] * d)[:d]
        var0 = p.get("var0", 0.25)
        f = np.empty((1, d, 2 ** n + 1))
        for i in range(d):
            x = _finest_nodes(p["lo"][i], p["hi"][i], n)
            f[0, i] = np.exp(-(x - mu0[i]) ** 2 / (2 * var0)) / math.sqrt(2 * math.pi * var0)
        p["mu0"] = mu0
        p["ic_w"], p["ic_f"] = np.ones(1), f
        return p
    f = np.zeros((1, d, 2 ** n + 1))
    f[0, :, 0] = 1.0
    p["ic_w"], p["ic_f"] = np.ones(1), f
    return p


# Workloads whose measurement needs tighter solver tolerances: in six
# dimensions the combination sums 1,709 grids with coefficients up to 10 in
# magnitude (sum of |c| = 7,183), so an error in the component states grows
# by about two orders of magnitude in the combined solution at the gather
# points, and the states must be solved well below 1e-10 for the gather to
# stay within 1e-8 of the oracle.
_TIGHT = {"varcoef6d": dict(tol=1e-12, mgrit_tol=1e-13)}


def metric_settings(prec: str, name: str | None = None) -> dict:
    """Solver tolerances of the throughput measurement: the final state and
    the combination at the gather points within 1e-8 relative L2 of the FP64
    oracle. Mixed: FP64-refined implicit steps to 1e-10 relative residual
    around FP32 inner solves to 1e-6; FP64: Krylov to 1e-10. Both: MGRIT
    C-point residual to 1e-9, and the implicit steps of the coarse MGRIT
    levels to 1e-3 (they only steer the correction, the fixed point is the
    fine-level one). The 6-D workload (`name`) solves its fine steps to
    1e-12 and MGRIT to 1e-13 (see _TIGHT)."""
    tight = _TIGHT.get(name, {})
    tol = tight.get("tol", 1e-10)
    mtol = tight.get("mgrit_tol", 1e-9)
    if prec == "mixed":
        return dict(prec="mixed", refine_tol=tol, inner_tol=1e-6, refine_maxit=12,
                    mgrit_tol=mtol, krylov_tol=1e-13, krylov_maxit=20000, mgrit_maxit=64,
                    coarse_tol=1e-3)
    return dict(prec="fp64", krylov_tol=tol, mgrit_tol=mtol, krylov_maxit=20000,
                mgrit_maxit=64, coarse_tol=1e-3)


def targets(p: dict, m: int, seed: int = 0) -> np.ndarray:
    """m seeded evaluation points in Omega, shape (m, d), float64.
    Lattice problems get integer lattice states 0..hi-1."""
    rng = np.random.default_rng(10_000 + seed)
    lo = np.asarray(p["lo"], dtype=np.float64)
    hi = np.asarray(p["hi"], dtype=np.float64)
    if p["op"] == "cme":
        return np.floor(rng.uniform(0.0, 1.0, size=(m, p["d"])) * (hi - lo) + lo)
    return lo + (hi - lo) * rng.uniform(0.0, 1.0, size=(m, p["d"]))


def random_vectors(length: int, count: int = 1, seed: int = 0) -> np.ndarray:
    """Seeded standard-normal test vectors of shape (count, length)."""
    rng = np.random.default_rng(20_000 + seed)
    return rng.standard_normal((count, length))
