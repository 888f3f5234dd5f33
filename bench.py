"""Benchmark of the batched mixed-precision MGRIT + combination solve on one
MI355X.

A step is one pass of the whole hot path over the workload: sampling of the
initial value on every component grid, MGRIT over the time interval on all
grids (FP32 Krylov inside FP64-refined implicit steps), and the FP64
combination gather at 1e5 seeded points. The default workload is the
largest one that fits one GPU: the 6-D variable-coefficient heat equation
u_t = div(a grad u), a = 1 + 0.5 prod sin(2 pi x_i), at sparse-grid level 8
(1,709 component grids, 849,161 unknowns per time level), 1,024
backward-Euler steps on [0, 0.1], three-level MGRIT with c = 8 and FCF
relaxation, CG.

Beside the timed path the line carries: the FP64 MGRIT path and batched
time-sequential stepping (both precisions) on the same workload, the plain
per-grid FP64 schedule (timed on a bounded number of steps and scaled), the
error of every path against the CPU oracle over all component grids, the
oracle itself timed on the host (one core on a grid sample; all allotted
cores on the whole workload), and the roofline of the dominant kernel.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
GATHER_POINTS = 100_000
METRIC = "DoF*timesteps/s + HBM GB/s, mixed vs FP64 GPU path at 1e-8 rel. L2 error"
# algorithmic HBM bytes of one implicit step per unknown: read the previous
# state, write the new one (FP64); every Krylov vector stays on chip
STEP_BYTES_PER_DOF = 16
# algorithmic HBM bytes per unknown of one streaming Krylov iteration with
# the vectors in HBM (FP64): CG fused apply+dot, fused update+dot, direction
# update = 40 B in FP32, doubled; BiCGStab twice that
STREAM_ALG_BYTES = {"cg": 80, "bicgstab": 160}
# what the wide streaming solver as built moves per unknown and iteration,
# summed over its kernels' passes (FP64 vectors, the five line-factor
# vectors in FP32: 20 B per preconditioner application). BiCGStab: the two
# line kernels read x, h, s, t, p, v + factors and x, h, r, v + factors and
# write x, r, p, h and x, s, h; the stencil kernels read h, r^ and h, s, r^
# and write v and t: 160 B read, 72 B written. CG: r + factors -> z;
# z, p -> p, q; x, p, r, q -> x, r: 76 B read, 40 B written.
STREAM_IMPL_BYTES = {"cg": 116, "bicgstab": 232}
# one-core oracle sample: every SAMPLE_STRIDE-th grid in canonical order
# (all layers of the index set), about 15 s of host work at the 6-D size
SAMPLE_STRIDE = 8
PLAIN_STEPS = 16  # steps of the plain per-grid schedule that are timed


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


OP_TEXT = {
    "heat": "heat equation u_t = Laplace(u)",
    "varcoef": "variable-coefficient heat equation u_t = div(a grad u), "
               "a = 1 + {amp} prod sin(2 pi x_i)",
    "ou": "Fokker-Planck equation of an Ornstein-Uhlenbeck process",
    "cme": "master equation of independent immigration-death species",
    "drift": "Fokker-Planck equation with a full drift matrix",
}


def describe(name: str, p: dict, G: int, slen: int) -> str:
    op = OP_TEXT[p["op"]].format(amp=p.get("amp", 0.0))
    lv = p["mgrit_levels"]
    mg = (f"{lv}-level MGRIT c={p['cf']} {p.get('relax', 'FCF')}" if lv > 1
          else "time-sequential stepping")
    prec = "mixed FP32/FP64" if p["prec"] == "mixed" else "FP64"
    return (f"{name}: {op}, d={p['d']}, sparse-grid level {p['n']} (L0={p.get('L0', 1)}), "
            f"{G} component grids, {slen} DoF per time level, {p['nsteps']} backward-Euler "
            f"steps on [{p['t0']},{p['t1']}], {mg}, {p['krylov'].upper()}, {prec}, gather at "
            f"{GATHER_POINTS} points")


def workload_problem(name: str, prec: str):
    """The workload with the solver tolerances of the measurement (final
    state within 1e-8 relative L2 of the FP64 oracle, reported as
    err_vs_oracle)."""
    from workloads import make, metric_settings
    p = make(name, prec=prec)
    p.update(metric_settings(prec, name))
    return p


def flops_per_iteration(d: int, krylov: str) -> int:
    # per unknown: CG = one (2d+1)-point apply (2(2d+1) flops) + 2 dots + 3 axpys;
    # BiCGStab = two applies + 4 dots + 6 axpys
    if krylov == "bicgstab":
        return 2 * 2 * (2 * d + 1) + 20
    return 2 * (2 * d + 1) + 10


def measured_traffic(workload: str, cls_key: str):
    """Calibrated HBM bytes per launch of a chain-kernel size class and
    precision ("W4K4/mixed") from the committed hardware-counter runs of this
    workload, or None once the kernel sources differ from the ones the
    counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "chain_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != workload:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["source_sha256"] or cls_key not in rec["classes"]:
        return None
    return rec["classes"][cls_key]["bytes_per_launch"]


def host_workers() -> int:
    """Host processes for the parallel oracle: the CPUs this process may run
    on, at most 16 (the share of the host that one GPU of the box gets)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_grids(prob, sel):
    from oracle import solve
    return sel, solve.component_states(prob, sel)


def _oracle_combine(prob, states, pts):
    from oracle import combine, solve
    return combine.combine_at(prob, solve.grid_list(prob), states, pts)


def _oracle_warm(_):
    from oracle import solve  # noqa: F401  (imports paid before the clock starts)
    return os.getpid()


def cpu_oracle_sample(prob, stride):
    """The oracle as it stands on one host core: time-sequential backward
    Euler with sparse LU on every stride-th component grid. Returns the
    seconds and the unknowns of the sample."""
    from oracle import solve
    gl = solve.grid_list(prob)
    sizes = np.diff(solve.offsets(prob))
    sel = list(range(0, len(gl), stride))
    t0 = time.perf_counter()
    solve.component_states(prob, sel)
    return time.perf_counter() - t0, int(sizes[sel].sum()), len(sel)


def cpu_oracle_parallel(prob, pts, workers):
    """The whole oracle (every grid, then the combination at the points)
    spread over `workers` host processes: the grids longest-first by
    unknowns, then the points. Started before the process touches the GPU;
    the worker start-up is outside the clock."""
    import concurrent.futures as cf
    import multiprocessing as mp
    from oracle import solve
    gl = solve.grid_list(prob)
    sizes = np.diff(solve.offsets(prob))
    bins = [[] for _ in range(workers)]
    load = [0] * workers
    for g in sorted(range(len(gl)), key=lambda g: -sizes[g]):
        b = load.index(min(load))
        bins[b].append(g)
        load[b] += int(sizes[g])
    bins = [b for b in bins if b]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_warm, range(4 * workers)))
        t0 = time.perf_counter()
        states = [None] * len(gl)
        for sel, st in ex.map(_oracle_grids, [prob] * len(bins), bins):
            for g, u in zip(sel, st):
                states[g] = u
        chunks = np.array_split(pts, workers)
        vals = np.concatenate(list(ex.map(_oracle_combine, [prob] * workers,
                                          [states] * workers, chunks)))
        t = time.perf_counter() - t0
    return t, workers, solve.packed(states), vals


# (d, n) cases of the manufactured heat family: two sparse-grid levels per d
# (levels 11 and up in 2-D and 3-D have grids beyond the on-chip size: they
# run on the streaming solvers, lines over 1,024 unknowns cut into segments)
MMS_CASES = [(2, 7), (2, 9), (2, 11), (2, 13), (2, 15), (3, 7), (3, 9), (3, 11), (3, 13),
             (4, 6), (4, 8), (4, 10), (5, 6), (5, 8), (6, 5), (6, 7)]


def mms_sweep(ctm, torch):
    """Section 4.2 family: heat equation on [0,1]^d with the manufactured
    solution, T = 1, N = 64 steps, two-level MGRIT with c = 2 and FCF,
    MGRIT tolerance 1e-8, mixed precision. Reports the MGRIT iterations (the
    paper observes them independent of d, L and the grid), the solve time
    and the error of the combination against u*(., T) at seeded points."""
    from workloads import make
    for d, n in MMS_CASES:
        p = make("heat_mms", d=d, n=n, nsteps=64, t1=1.0)
        p.update(prec="mixed", refine_tol=1e-10, inner_tol=1e-6, refine_maxit=12,
                 mgrit_tol=1e-8, krylov_tol=1e-13, krylov_maxit=20000, mgrit_maxit=64,
                 coarse_tol=1e-3)
        plan = ctm.Plan(p)
        u = plan.solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        u = plan.solve()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        st = plan.stats()
        rng = np.random.default_rng(3)
        pts = rng.uniform(0.05, 0.95, size=(2000, d))
        got = plan.gather(u, torch.from_numpy(pts).cuda()).cpu().numpy()
        r = np.sqrt(np.sum(pts * pts, axis=1) + 1.0)
        exact = r * np.exp(-1.0) * np.prod(np.sin(np.pi * pts), axis=1)
        print(json.dumps(dict(case="heat_mms", d=d, n=n, grids=plan.G, dof_per_level=plan.slen,
                              nsteps=64, mgrit_iterations=st["mgrit_iterations"], ms=round(ms, 2),
                              krylov_iterations=st["krylov_iterations"],
                              max_error_vs_exact=float(np.abs(got - exact).max()))), flush=True)
    return 0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _per_grid_max_rel(prob, a, b):
    """Largest relative L2 error of one component grid."""
    from oracle import solve
    off = solve.offsets(prob)
    worst = 0.0
    for g in range(len(off) - 1):
        x, y = a[off[g]:off[g + 1]], b[off[g]:off[g + 1]]
        worst = max(worst, float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)))
    return worst


def _errors(prob, u, oracle_u):
    if oracle_u is None:
        return {}
    return {"state_rel_l2_vs_oracle": _rel(u, oracle_u),
            "max_grid_rel_l2_vs_oracle": _per_grid_max_rel(prob, u, oracle_u)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _shapes(args, plan):
    """Launch shapes of the timed plan, outside the timed region: autotuned
    (ctm_autotune), taken from a file, or the defaults."""
    if args.load_shapes:
        with open(args.load_shapes) as f:
            rec = json.load(f)
        assert rec["workload"] == args.workload and len(rec["shapes"]) == plan.G
        for g, (w, k) in enumerate(rec["shapes"]):
            if k:
                plan.set_grid_shape(g, w, k)
        return {"source": args.load_shapes}
    tune = None
    if args.tune:
        tune = plan.autotune(trial_iterations=2, repeats=1)
        log(f"autotune: {tune}")
    if args.save_shapes:
        with open(args.save_shapes, "w") as f:
            json.dump({"workload": args.workload,
                       "shapes": [plan.grid_shape(g) for g in range(plan.G)]}, f)
    return tune


def _timed(torch, fn, reps=1):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def _comparators(args, ctm, torch, oracle_u, dof_steps):
    """FP64 MGRIT at the measurement's tolerances, batched
    time-sequential stepping (mixed and FP64), and the plain per-grid FP64
    schedule on the same workload, outside the timed region, each with its
    error against the oracle. The plain schedule launches one kernel per
    grid and step; it is timed on PLAIN_STEPS steps and scaled to N."""
    out = {}
    runs = [
        ("fp64_mgrit", workload_problem(args.workload, "fp64"), "solve"),
        ("mixed_sequential_batched", dict(workload_problem(args.workload, "mixed"),
                                          mgrit_levels=1), "solve"),
        ("fp64_sequential_batched", dict(workload_problem(args.workload, "fp64"),
                                         mgrit_levels=1), "solve"),
        ("fp64_per_grid_plain", workload_problem(args.workload, "fp64"), "per_grid"),
    ]
    for name, prob, kind in runs:
        plan = ctm.Plan(prob)
        entry = {"tolerances": {k: prob.get(k) for k in ("krylov_tol", "mgrit_tol", "coarse_tol",
                                                          "refine_tol", "inner_tol")}}
        if kind == "solve":
            sec, u = _timed(torch, lambda: plan.solve(), reps=2)
            st = plan.stats()
            entry.update(seconds=sec, value=dof_steps / sec,
                         mgrit_iterations=st["mgrit_iterations"],
                         krylov_iterations=st["krylov_iterations"],
                         phi_solves=st["phi_solves"])
            entry.update(_errors(prob, u.cpu().numpy(), oracle_u))
        else:
            u0 = plan.initial_state()
            n = min(PLAIN_STEPS, prob["nsteps"])
            sec, _ = _timed(torch, lambda: plan.propagate(u0, n, per_grid=True))
            scaled = sec * prob["nsteps"] / n
            entry.update(seconds=scaled, value=dof_steps / scaled, timed_steps=n,
                         timed_seconds=sec, launches=plan.G * n,
                         note=f"one launch per grid and step; {n} of {prob['nsteps']} steps "
                              "timed, scaled linearly")
        out[name] = entry
        log(f"{name}: {entry['seconds'] * 1e3:.1f} ms ({entry['value']:.3e} DoF*steps/s)")
        del plan
    return out


def _copy_calibration(torch):
    """A plain 256 MiB device copy, the last kernel of a counter run: its
    FETCH_SIZE / WRITE_SIZE counts calibrate the kernels' ones."""
    src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return {"read": src.numel() * 8, "write": dst.numel() * 8}


def copy_bandwidth(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (GB/s, read + write bytes) of a
    plain 1 GiB copy: the practical HBM ceiling beside the 8 TB/s peak."""
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2.0 * n * 8 / sec / 1e9


def _streaming(ctm, torch):
    """The streaming solvers on grids beyond the on-chip solver: the 2-D
    oscillator of Section 4.4 at the paper's own levels (L = 14, L0 = 6:
    seven grids of up to 32,193 unknowns), FP64 MGRIT. Their roofline is
    HBM. Algorithmic bytes (the streaming BiCGStab iteration: 160 B per
    unknown in FP64) and the bytes the solver as built moves (232 B: the
    line-factor vectors of the preconditioner besides the Krylov sweeps),
    both over the wall time of the solve and over the wide solver's own
    launch time (a wide launch is its whole chain, host polls included)."""
    from workloads import make
    p = make("fp_osc2d", n=14, L0=6, prec="fp64")
    # the measurement tolerances of the main workload (coarse levels to 1e-3)
    p.update(krylov_tol=1e-10, mgrit_tol=1e-9, mgrit_maxit=64, krylov_maxit=20000,
             coarse_tol=1e-3)
    plan = ctm.Plan(p)
    plan.solve()
    torch.cuda.synchronize()
    plan.set_timing(True)
    t0 = time.perf_counter()
    plan.solve()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    st = plan.stats()
    plan.set_timing(False)
    alg = STREAM_ALG_BYTES[p["krylov"]]
    impl = STREAM_IMPL_BYTES[p["krylov"]]
    wide = [c for c in st["shapes"] if c["K"] == 0 and c["W"] == 4]
    if not wide:
        return None
    c = wide[0]
    copy_gbps = copy_bandwidth(torch)
    launch_s = c["ms"] / 1e3
    achieved = c["work"] * alg / launch_s / 1e9 if launch_s > 0 else None
    return {
        "workload": f"fp_osc2d at L = 14, L0 = 6: {plan.G} grids, {plan.slen} DoF per level, "
                    f"{p['nsteps']} steps, 2-level MGRIT c = 2, BiCGStab, FP64, Krylov 1e-10, "
                    f"coarse levels 1e-3, MGRIT 1e-9",
        "seconds": sec,
        "value": plan.slen * p["nsteps"] / sec,
        "mgrit_iterations": st["mgrit_iterations"],
        "krylov_iterations": st["krylov_iterations"],
        "roofline": {
            "kernel": "wide solver: many work-groups per task, one launch per Krylov phase "
                      "for all tasks of a launch",
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS if achieved else None,
            "bytes_per_unknown_iteration": alg,
            "implementation_bytes_per_unknown_iteration": impl,
            "implementation_GBps": c["work"] * impl / launch_s / 1e9 if launch_s > 0 else None,
            "algorithmic_GBps_over_solve_wall": c["work"] * alg / sec / 1e9,
            "wide_launch_ms": c["ms"], "krylov_work": c["work"],
            "copy_GBps": copy_gbps,
            "frac_of_copy": achieved / copy_gbps if achieved else None,
        },
    }


def _residual_mode(ctm, torch):
    """The optimized oscillator run of Section 4.4 (T = 1, N = 3204, c = 12,
    F-relaxation, tolerance 1e-4): MGRIT in space-time residual mode with two
    Krylov iterations per step, beside the same MGRIT with every step solved
    to 1e-10. Solve time (second of two solves) and MGRIT iterations."""
    from workloads import make
    out = {}
    for tag, kw in (("residual_mode_2_iterations", dict(residual_mode=1, krylov_maxit=2)),
                    ("exact_steps", dict(residual_mode=0, krylov_maxit=20000,
                                         krylov_tol=1e-10))):
        p = make("fp_osc2d", t1=1.0, nsteps=3204)
        p.update(cf=12, relax="F", prec="fp64", mgrit_tol=1e-4, mgrit_maxit=100, **kw)
        plan = ctm.Plan(p)
        sec, _ = _timed(torch, lambda: plan.solve())
        st = plan.stats()
        out[tag] = {"seconds": sec, "mgrit_iterations": st["mgrit_iterations"],
                    "krylov_iterations": st["krylov_iterations"]}
    return out


def _heat3d(ctm, torch):
    """The 3-D heat workload (109 grids, 73,915 unknowns per level, 256 steps,
    two-level MGRIT c = 8) at the measurement's settings: solve times of the
    mixed and FP64 MGRIT paths and the mixed path's error against the
    oracle."""
    from oracle import solve
    out = {}
    ref = None
    for prec in ("mixed", "fp64"):
        p = workload_problem("heat3d", prec)
        if ref is None:
            ref = solve.packed(solve.component_states(p))
        plan = ctm.Plan(p)
        sec, u = _timed(torch, lambda: plan.solve(), reps=3)
        st = plan.stats()
        out[f"{prec}_mgrit"] = {"seconds": sec, "value": plan.slen * p["nsteps"] / sec,
                                "mgrit_iterations": st["mgrit_iterations"],
                                **_errors(p, u.cpu().numpy(), ref)}
    return out


def _table3_ct(ctm, torch):
    """Section 4.4.1's time-sequential combination run (Table 3, CT): the 2-D
    oscillator on L = 14, L0 = 6 (seven grids, 177,415 unknowns per level),
    20,000 backward-Euler steps of 0.005 to T = 100, FP64 BiCGStab with the
    line preconditioner to 1e-10, every grid on the wide streaming solver.
    One solve after a short warm-up; the paper's figure for the same scheme
    is 1,326 s on 176 cores of its CPU cluster (context, not a target)."""
    from workloads import make
    p = make("fp_osc2d", n=14, L0=6, prec="fp64")
    p.update(t1=100.0, nsteps=20000, mgrit_levels=1, krylov_tol=1e-10, krylov_maxit=20000)
    plan = ctm.Plan(p)
    u0 = plan.initial_state()
    plan.propagate(u0, 40)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    st = plan.stats()
    return {"seconds": sec, "steps": p["nsteps"], "value": plan.slen * p["nsteps"] / sec,
            "krylov_iterations": st["krylov_iterations"],
            "paper_ct_seconds_176_cores": 1326.0}


def _schwarz(ctm, torch):
    """The paper's spatial preconditioner (Section 2.1.2) beside the line
    preconditioner on the 3-D heat workload in FP64 at the measurement's
    tolerances: solve time, MGRIT and Krylov iterations. With Schwarz every
    grid runs on the streaming solver (one 1,024-thread work-group per task,
    vectors in HBM), balanced form with CG, subdomains of 2^5 unknowns."""
    out = {}
    for tag, kw in (("line", {}), ("schwarz_S5", dict(precond="schwarz", schwarz_s=5))):
        p = workload_problem("heat3d", "fp64")
        p.update(kw)
        plan = ctm.Plan(p)
        sec, _ = _timed(torch, lambda: plan.solve(), reps=2)
        st = plan.stats()
        out[tag] = {"seconds": sec, "mgrit_iterations": st["mgrit_iterations"],
                    "krylov_iterations": st["krylov_iterations"],
                    "krylov_per_solve": st["krylov_iterations"] / max(1, st["phi_solves"])}
        del plan
    return out


def _roofline(shapes, d, krylov, prec, copy_gbps):
    """Roofline of the dominant kernel: the size class of the implicit-step
    kernel with the most device time. Its algorithmic HBM bytes are 16 B per
    unknown and implicit step (read the previous state, write the new one);
    the FP32/FP64 flops of its Krylov iterations are reported beside."""
    # on-chip size classes only (K > 0): not the streaming solvers, nor the
    # FP64 coarse-level launches of a mixed plan, which are reported apart
    (dw, dk), dom = max(((k, v) for k, v in shapes.items() if k[1] > 0),
                        key=lambda kv: kv[1]["ms"])
    dom_s = dom["ms"] / 1e3
    nl = max(dom["launches"], 1)
    alg_bytes = STEP_BYTES_PER_DOF * dom["dofsteps"]
    achieved = alg_bytes / dom_s / 1e9 if dom_s > 0 else None
    fpi = flops_per_iteration(d, krylov)
    tflops = dom["work"] * fpi / dom_s / 1e12 if dom_s > 0 else None
    peak_f = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
    return (dw, dk), {
        "kernel": f"chain_kernel W={dw} K={dk} (batched implicit steps of one size class: "
                  f"{'FP32 preconditioned ' if prec == 'mixed' else 'FP64 preconditioned '}"
                  f"{krylov.upper()} on chip{' inside FP64 refinement' if prec == 'mixed' else ''})",
        "bound": "hbm",
        "achieved": achieved,
        "peak": PEAK_HBM_GBPS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBPS if achieved else None,
        "traffic": None,
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "avg_launch_ms": dom["ms"] / nl,
        "launches": dom["launches"],
        "bytes_per_dof_step": STEP_BYTES_PER_DOF,
        "dof_steps_per_launch": dom["dofsteps"] / nl,
        "algorithmic_bytes_per_launch": alg_bytes / nl,
        "vector_role_bytes_per_launch": dom["bytes"] / nl,
        "krylov_flops": {"achieved_TFLOPs": tflops, "peak_TFLOPs": peak_f,
                         "frac": tflops / peak_f if tflops else None,
                         "flops_per_unknown_iteration": fpi,
                         "note": "vector peak; the on-chip Krylov iteration is bound by "
                                 "latency (occupancy, barriers, reductions)"},
        "copy_GBps": copy_gbps,
        "all_classes": {("fp64_coarse_levels" if (w, k) == (0, 0) else f"W{w}K{k}"): v
                        for (w, k), v in sorted(shapes.items())},
    }


def summarize_traffic(workload: str, fetch_dir: str, write_dir: str, out_path: str):
    """Calibrated HBM bytes per launch of every chain-kernel size class from
    two rocprofv3 counter runs of `bench.py --copy-calibration` (FETCH_SIZE,
    then WRITE_SIZE; KiB per dispatch). The run ends with a plain copy of a
    known size, which gives the factor from each counter to bytes. Writes the
    record `measured_traffic` reads, keyed by the kernel sources' hash."""
    import csv
    import hashlib
    import re
    sources = ["paper_2509_22156_amd/csrc/chain_kernel.hpp",
               "paper_2509_22156_amd/csrc/line_layout.hpp",
               "paper_2509_22156_amd/csrc/device_common.hpp",
               "paper_2509_22156_amd/csrc/ctm_internal.h"]
    copy_bytes = 32 * 2 ** 20 * 8

    def per_dispatch(d, counter):
        rows = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            rows.setdefault(key, [r["Kernel_Name"], 0.0])
            rows[key][1] += float(r["Counter_Value"])
        return [rows[k] for k in sorted(rows)]

    def classes(rows):
        acc = {}
        for name, kib in rows:
            m = re.search(r"chain_kernel<\d+, \d+, (true|false), \d+, (\d+), (\d+)>", name)
            if m:
                prec = "mixed" if m.group(1) == "true" else "fp64"
                a = acc.setdefault(f"W{m.group(2)}K{m.group(3)}/{prec}", [0.0, 0])
                a[0] += kib
                a[1] += 1
        return acc

    def copy_kib(rows):
        # the calibration copy is the last dispatch of the run
        return rows[-1][1]
    fetch = per_dispatch(fetch_dir, "FETCH_SIZE")
    write = per_dispatch(write_dir, "WRITE_SIZE")
    rf = copy_bytes / (copy_kib(fetch) * 1024.0)
    wf = copy_bytes / (copy_kib(write) * 1024.0)
    cf, cw = classes(fetch), classes(write)
    rec_classes = {}
    for k in sorted(cf):
        n = cf[k][1]
        rec_classes[k] = {"dispatches": n,
                          "fetch_kib_per_launch": cf[k][0] / n,
                          "write_kib_per_launch": cw[k][0] / cw[k][1],
                          "bytes_per_launch": (cf[k][0] / n * rf + cw[k][0] / cw[k][1] * wf) * 1024.0}
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    rec = {"workload": workload, "source_sha256": h.hexdigest(), "sources": sources,
           "read_factor": rf, "write_factor": wf, "copy_bytes": copy_bytes,
           "classes": rec_classes}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="varcoef6d")
    ap.add_argument("--no-extras", action="store_true", help="skip the comparator runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mms-sweep", action="store_true",
                    help="instead of the metric: the manufactured heat family of Section 4.2 "
                         "over d = 2..6 and two levels each (one JSON line per case)")
    ap.add_argument("--streaming-only", action="store_true",
                    help="instead of the metric: only the streaming-kernel workload (the "
                         "paper-size 2-D oscillator), one JSON line")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch shapes before timing (ctm_autotune)")
    ap.add_argument("--save-shapes", default=None,
                    help="write the launch shape of every grid to this JSON file")
    ap.add_argument("--load-shapes", default=None,
                    help="take the launch shapes from this JSON file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 256 MiB device copy (hardware-counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="instead of the metric: summarise two rocprofv3 counter runs "
                         "(FETCH_SIZE, WRITE_SIZE) of --copy-calibration into "
                         "profiles/chain_kernel_traffic.json")
    args = ap.parse_args(argv)

    if args.traffic_from:
        rec = summarize_traffic(args.workload, *args.traffic_from,
                                os.path.join(ROOT, "profiles", "chain_kernel_traffic.json"))
        print(json.dumps(rec))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (it would "
              "shard by component grid, with one all-reduce of the combined target vector per "
              "recombination step)", file=sys.stderr)
        return 2

    from workloads import targets
    par = None
    if not (args.mms_sweep or args.streaming_only):
        prob = workload_problem(args.workload, "mixed")
        if not args.no_cpu:
            # the parallel oracle runs first: its worker processes start
            # before this process loads the HIP library or touches the GPU
            workers = host_workers()
            log(f"cpu baseline: the whole oracle over {workers} host processes")
            par = cpu_oracle_parallel(prob, targets(prob, GATHER_POINTS, seed=0), workers)
            log(f"parallel oracle {par[0]:.2f} s on {par[1]} processes")

    import torch
    from paper_2509_22156_amd import ctm

    torch.cuda.set_device(0)
    if args.mms_sweep:
        return mms_sweep(ctm, torch)
    if args.streaming_only:
        out = _streaming(ctm, torch)
        if args.copy_calibration:
            out["copy_calibration_bytes"] = _copy_calibration(torch)
        print(json.dumps(out), flush=True)
        return 0
    t0 = time.perf_counter()
    plan = ctm.Plan(prob)
    plan_ms = (time.perf_counter() - t0) * 1e3
    tune = _shapes(args, plan)
    pts_np = targets(prob, GATHER_POINTS, seed=0)
    pts = torch.from_numpy(pts_np).cuda()
    u = torch.empty(plan.slen, dtype=torch.float64, device="cuda")
    vals = torch.empty(GATHER_POINTS, dtype=torch.float64, device="cuda")
    plan.workspace()
    N = prob["nsteps"]
    dof_steps = plan.slen * N
    log(f"workload {args.workload}: G={plan.G} dof/level={plan.slen} N={N} "
        f"ws={plan.workspace_bytes / 2**20:.1f} MiB")

    def step():
        plan.solve(out=u)
        plan.gather(u, pts, out=vals)

    plan.set_timing(False)
    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    plan.set_timing(True)
    agg = dict(chain_ms=0.0, chain_launches=0, krylov_work=0, chain_bytes=0.0,
               mgrit_iterations=0, krylov_iterations=0, phi_solves=0, refine_sweeps=0)
    shapes = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        st = plan.stats()
        for k in agg:
            agg[k] += st[k]
        for sh in st["shapes"]:
            key = (sh["W"], sh["K"])
            acc = shapes.setdefault(key, dict(ms=0.0, launches=0, work=0, bytes=0.0, dofsteps=0))
            for k in acc:
                acc[k] += sh[k]
        log(f"step {i + 1}/{args.steps}: mgrit it={st['mgrit_iterations']} "
            f"res={st['mgrit_residual'][-1]:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.set_timing(False)
    ms_per_step = elapsed * 1e3 / args.steps
    value = dof_steps / (elapsed / args.steps)
    copy_gbps = copy_bandwidth(torch)  # measured after the timed steps
    (dw, dk), roofline = _roofline(shapes, prob["d"], prob["krylov"], prob["prec"], copy_gbps)
    roofline["traffic"] = measured_traffic(args.workload, f"W{dw}K{dk}/{prob['prec']}")
    u_mixed = u.cpu().numpy()
    vals_mixed = vals.cpu().numpy()
    log(f"mixed MGRIT: {ms_per_step:.2f} ms/step, {value:.3e} DoF*steps/s, dominant W{dw}K{dk} "
        f"{roofline['avg_launch_ms']:.3f} ms/launch, {roofline['achieved']:.1f} GB/s")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF*timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": describe(args.workload, prob, plan.G, plan.slen),
            "grids": plan.G, "dof_per_level": plan.slen, "nsteps": N,
            "tolerances": {k: prob.get(k) for k in ("refine_tol", "inner_tol", "mgrit_tol",
                                                     "coarse_tol")},
            "mgrit_iterations_per_step": agg["mgrit_iterations"] / args.steps,
            "phi_solves_per_step": agg["phi_solves"] / args.steps,
            "krylov_iterations_per_step": agg["krylov_iterations"] / args.steps,
            "refine_sweeps_per_step": agg["refine_sweeps"] / args.steps,
            "plan_ms": plan_ms,
            "autotune": tune,
        },
        "roofline": roofline,
    }

    oracle_u = oracle_vals = None
    if par is not None:
        oracle_u, oracle_vals = par[2], par[3]
        result["err_vs_oracle"] = {
            "grids_compared": plan.G,
            "mixed_state_rel_l2": _rel(u_mixed, oracle_u),
            "mixed_max_grid_rel_l2": _per_grid_max_rel(prob, u_mixed, oracle_u),
            "mixed_gather_rel_l2": _rel(vals_mixed, oracle_vals),
        }
        log(f"mixed error vs oracle {result['err_vs_oracle']}")
        log("cpu baseline: oracle on one host core (grid sample)")
        t_cpu, dof_sample, nsample = cpu_oracle_sample(prob, SAMPLE_STRIDE)
        result["cpu_baseline"] = {
            "value": dof_sample * N / t_cpu,
            "unit": "DoF*timesteps/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"every {SAMPLE_STRIDE}th component grid ({nsample} of {plan.G} grids, "
                      f"{dof_sample} of {plan.slen} DoF per level, all layers) x {N} steps, "
                      f"sparse LU, single thread; {t_cpu:.2f} s",
            "cpu": _cpu_model(),
        }
        result["cpu_baseline_parallel"] = {
            "value": dof_steps / par[0],
            "unit": "DoF*timesteps/s",
            "cores": par[1],
            "kind": "oracle",
            "sample": f"whole workload over {par[1]} host processes (the CPUs allotted to this "
                      f"process, at most 16): grids longest-first, then the {GATHER_POINTS} "
                      f"combination points; {par[0]:.2f} s",
            "cpu": _cpu_model(),
        }

    if not args.no_extras:
        comp = _comparators(args, ctm, torch, oracle_u, dof_steps)
        result["comparators"] = comp
        # the whole timed step (solve + gather) against the other paths' solves
        step_s = ms_per_step / 1e3
        result["speedup_vs_plain_per_grid_fp64"] = comp["fp64_per_grid_plain"]["seconds"] / step_s
        result["speedup_vs_fp64_mgrit"] = comp["fp64_mgrit"]["seconds"] / step_s
        result["speedup_vs_fp64_sequential_batched"] = (
            comp["fp64_sequential_batched"]["seconds"] / step_s)
        result["streaming"] = _streaming(ctm, torch)
        log(f"streaming: {result['streaming']}")
        result["residual_mode"] = _residual_mode(ctm, torch)
        log(f"residual mode: {result['residual_mode']}")
        if args.workload != "heat3d":
            result["heat3d"] = _heat3d(ctm, torch)
            log(f"heat3d: {result['heat3d']}")
        result["schwarz_vs_line"] = _schwarz(ctm, torch)
        log(f"schwarz vs line: {result['schwarz_vs_line']}")
        result["table3_ct"] = _table3_ct(ctm, torch)
        log(f"table 3 CT: {result['table3_ct']}")
    if args.copy_calibration:
        result["copy_calibration_bytes"] = _copy_calibration(torch)

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
