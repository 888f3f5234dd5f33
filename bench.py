"""Benchmark of the batched mixed-precision MGRIT + combination solve on one
MI355X.

A step is one pass of the whole hot path over the workload: sampling of the
initial value on every component grid, MGRIT over the time interval on all
grids (FP32 Krylov inside FP64-refined implicit steps), and the FP64
combination gather at 1e5 seeded points. The workload is the 3-D heat
equation at sparse-grid level 9 (109 component grids, 73,915 unknowns per
time level, 256 backward-Euler steps on [0, 0.05], two-level MGRIT with
c = 8).

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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_problem(name: str, prec: str):
    """The workload with the solver tolerances of the measurement (final
    state within 1e-8 relative L2 of the FP64 oracle, reported as
    err_vs_oracle)."""
    from workloads import make, metric_settings
    p = make(name, prec=prec)
    p.update(metric_settings(prec))
    return p


def flops_per_iteration(d: int, krylov: str) -> int:
    # per unknown: CG = one (2d+1)-point apply (2(2d+1) flops) + 2 dots + 3 axpys;
    # BiCGStab = two applies + 4 dots + 6 axpys
    if krylov == "bicgstab":
        return 2 * 2 * (2 * d + 1) + 20
    return 2 * (2 * d + 1) + 10


def measured_traffic(cls_key: str):
    """Calibrated HBM bytes per launch of a chain-kernel size class from the
    committed hardware-counter runs, or None once the kernel sources differ
    from the ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "chain_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["source_sha256"] or cls_key not in rec["classes"]:
        return None
    return rec["classes"][cls_key]["bytes_per_launch"]


def cpu_oracle(prob, pts):
    """The oracle as it stands on this host: time-sequential backward Euler
    with sparse LU on every grid, then the combination at the points."""
    from oracle import combine, solve
    t0 = time.perf_counter()
    states = solve.component_states(prob)
    vals = combine.combine_at(prob, solve.grid_list(prob), states, pts)
    return time.perf_counter() - t0, solve.packed(states), vals


def _oracle_grids(prob, sel):
    from oracle import solve
    return sel, solve.component_states(prob, sel)


def _oracle_combine(prob, states, pts):
    from oracle import combine, solve
    return combine.combine_at(prob, solve.grid_list(prob), states, pts)


def _oracle_warm(_):
    from oracle import solve  # noqa: F401  (imports paid before the clock starts)
    return os.getpid()


def cpu_oracle_parallel(prob, pts, workers):
    """The same oracle spread over `workers` host processes: the grids
    (longest-first by unknowns), then the points of the combination. Started
    before the process touches the GPU; the worker start-up is outside the
    clock."""
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
    return t, max(len(bins), workers), solve.packed(states), vals


# (d, n) cases of the manufactured heat family: two sparse-grid levels per d
MMS_CASES = [(2, 7), (2, 9), (3, 7), (3, 9), (4, 6), (4, 8), (5, 6), (5, 8), (6, 5), (6, 7)]


def mms_sweep(ctm, torch):
    """Section 4.2 family: heat equation on [0,1]^d with the manufactured
    solution, T = 1, N = 64 steps, two-level MGRIT with c = 2 and FCF,
    MGRIT tolerance 1e-8, mixed precision. Reports the MGRIT iterations (the
    paper observes them independent of d, L and the grid), the solve time
    and the error of the combination against u*(., T) at seeded points."""
    import numpy as np
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat3d")
    ap.add_argument("--no-extras", action="store_true", help="skip the comparator runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mms-sweep", action="store_true",
                    help="instead of the metric: the manufactured heat family of Section 4.2 "
                         "over d = 2..6 and two levels each (one JSON line per case)")
    ap.add_argument("--streaming-only", action="store_true",
                    help="instead of the metric: only the streaming-kernel workload (the "
                         "paper-size 2-D oscillator), one JSON line")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the plan's default launch shapes (no autotuning)")
    ap.add_argument("--save-shapes", default=None,
                    help="write the tuned launch shape of every grid to this JSON file")
    ap.add_argument("--load-shapes", default=None,
                    help="take the launch shapes from this JSON file instead of tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a plain 256 MiB device copy (hardware-counter calibration)")
    args = ap.parse_args(argv)

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
            workers = max(1, min(16, os.cpu_count() or 1))
            log(f"cpu baseline: oracle over {workers} host processes")
            par = cpu_oracle_parallel(prob, targets(prob, GATHER_POINTS, seed=0), workers)
            log(f"parallel oracle {par[0]:.2f} s on {par[1]} processes")

    import torch
    from paper_2509_22156_amd import ctm

    if args.mms_sweep:
        torch.cuda.set_device(0)
        return mms_sweep(ctm, torch)
    if args.streaming_only:
        torch.cuda.set_device(0)
        print(json.dumps(_streaming(ctm, torch)), flush=True)
        return 0
    torch.cuda.set_device(0)
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
            acc = shapes.setdefault(key, dict(ms=0.0, launches=0, work=0, bytes=0.0))
            acc["ms"] += sh["ms"]
            acc["launches"] += sh["launches"]
            acc["work"] += sh["work"]
            acc["bytes"] += sh["bytes"]
        log(f"step {i + 1}/{args.steps}: mgrit it={st['mgrit_iterations']} "
            f"res={st['mgrit_residual'][-1]:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.set_timing(False)
    ms_per_step = elapsed * 1e3 / args.steps
    value = dof_steps / (elapsed / args.steps)

    d = prob["d"]
    fpi = flops_per_iteration(d, prob["krylov"])
    chain_s = agg["chain_ms"] / 1e3
    # dominant kernel: the size class of the implicit-step kernel with the
    # most device time; its algorithmic FP32 flops over its own timed launches
    (dw, dk), dom = max(shapes.items(), key=lambda kv: kv[1]["ms"])
    dom_s = dom["ms"] / 1e3
    achieved_tflops = dom["work"] * fpi / dom_s / 1e12 if dom_s > 0 else None
    launches = max(agg["chain_launches"], 1)
    roofline = {
        "kernel": f"chain_kernel<heat, CG, mixed, W={dw}, K={dk}> (batched implicit steps, "
                  "FP32 preconditioned CG inside FP64 refinement)",
        "bound": "alu",
        "achieved": achieved_tflops,
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": (achieved_tflops / PEAK_FP32_TFLOPS) if achieved_tflops else None,
        "traffic": measured_traffic(f"W{dw}K{dk}"),
        "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "avg_launch_ms": dom["ms"] / max(dom["launches"], 1),
        "launches": dom["launches"],
        "algorithmic_flops_per_launch": dom["work"] * fpi / max(dom["launches"], 1),
        "algorithmic_bytes_per_launch": dom["bytes"] / max(dom["launches"], 1),
        "all_classes": {f"W{w}K{k}": v for (w, k), v in sorted(shapes.items())},
        "phase_ms_per_step": agg["chain_ms"] / args.steps,
        "algorithmic_hbm_GBps": agg["chain_bytes"] / chain_s / 1e9 if chain_s > 0 else None,
        "hbm_frac": (agg["chain_bytes"] / chain_s / 1e9 / PEAK_HBM_GBPS) if chain_s > 0 else None,
        "copy_GBps": copy_bandwidth(torch),  # measured after the timed steps
    }
    u_mixed = u.cpu().numpy()
    vals_mixed = vals.cpu().numpy()
    it_per_step = agg["mgrit_iterations"] / args.steps
    log(f"mixed MGRIT: {ms_per_step:.2f} ms/step, {value:.3e} DoF*steps/s, "
        f"chain {agg['chain_ms'] / args.steps:.2f} ms/step in {launches // args.steps} launches")

    result = {
        "metric": "DoF*timesteps/s (mixed FP32/FP64 batched MGRIT + combination)",
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
            "workload": f"{args.workload}: heat equation d={d}, sparse-grid level {prob['n']}, "
                        f"{plan.G} component grids, {plan.slen} DoF per time level, {N} "
                        f"backward-Euler steps on [0,{prob['t1']}], {prob['mgrit_levels']}-level "
                        f"MGRIT c={prob['cf']} FCF, CG, mixed precision, gather at "
                        f"{GATHER_POINTS} points",
            "grids": plan.G, "dof_per_level": plan.slen, "nsteps": N,
            "mgrit_iterations_per_step": it_per_step,
            "phi_solves_per_step": agg["phi_solves"] / args.steps,
            "krylov_iterations_per_step": agg["krylov_iterations"] / args.steps,
            "plan_ms": plan_ms,
            "autotune": tune,
        },
        "roofline": roofline,
    }

    oracle_u = oracle_vals = None
    if not args.no_cpu:
        log("cpu baseline: oracle on the host")
        t_cpu, oracle_u, oracle_vals = cpu_oracle(prob, pts_np)
        result["cpu_baseline"] = {
            "value": dof_steps / t_cpu,
            "unit": "DoF*timesteps/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"whole workload ({plan.G} grids x {N} steps, sparse LU, single thread) "
                      f"+ combination at {GATHER_POINTS} points; {t_cpu:.2f} s",
            "cpu": _cpu_model(),
        }
        if par is not None:
            result["cpu_baseline_parallel"] = {
                "value": dof_steps / par[0],
                "unit": "DoF*timesteps/s",
                "cores": par[1],
                "kind": "oracle",
                "sample": f"whole workload over {par[1]} host processes: grids longest-first, "
                          f"then the {GATHER_POINTS} combination points; {par[0]:.2f} s",
            }
            assert _rel(par[2], oracle_u) == 0.0
        result["err_vs_oracle"] = {
            "mixed_state_rel_l2": _rel(u_mixed, oracle_u),
            "mixed_gather_rel_l2": _rel(vals_mixed, oracle_vals),
        }
        log(f"cpu {t_cpu:.2f} s; mixed err {result['err_vs_oracle']}")

    if not args.no_extras:
        result["comparators"] = _comparators(args, ctm, torch, oracle_u, dof_steps)
        plain = result["comparators"]["fp64_per_grid_plain"]["seconds"]
        # the whole timed step (solve + gather) against the plain schedule's solve
        result["speedup_vs_plain_per_grid_fp64"] = plain / (ms_per_step / 1e3)
        result["streaming"] = _streaming(ctm, torch)
        result["residual_mode"] = _residual_mode(ctm, torch)
        log(f"residual mode: {result['residual_mode']}")
        log(f"streaming: {result['streaming']}")
    if args.copy_calibration:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 8, "write": dst.numel() * 8}

    print(json.dumps(result), flush=True)
    return 0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


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
    (ctm_autotune, full trial solves, fastest of two), taken from a file, or
    the defaults."""
    if args.load_shapes:
        with open(args.load_shapes) as f:
            rec = json.load(f)
        assert rec["workload"] == args.workload and len(rec["shapes"]) == plan.G
        for g, (w, k) in enumerate(rec["shapes"]):
            if k:
                plan.set_grid_shape(g, w, k)
        return {"source": args.load_shapes}
    tune = None
    if not args.no_tune:
        tune = plan.autotune(trial_iterations=0, repeats=2)
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
    """FP64 MGRIT, batched time-sequential stepping (mixed and FP64) and the
    plain per-grid FP64 schedule on the same workload, outside the timed
    region, each with its error against the oracle. The batched ones are
    autotuned like the timed plan (unless --no-tune) and timed as the mean
    of three solves; the plain schedule keeps the default shapes."""
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
        u0 = plan.initial_state()
        if kind == "solve":
            if not args.no_tune:
                plan.autotune(trial_iterations=0, repeats=2)
            sec, u = _timed(torch, lambda: plan.solve(), reps=3)
            st = plan.stats()
        else:
            sec, u = _timed(torch, lambda: plan.propagate(u0, prob["nsteps"], per_grid=True))
            st = plan.stats()
        entry = {"seconds": sec, "value": dof_steps / sec,
                 "mgrit_iterations": st["mgrit_iterations"],
                 "krylov_iterations": st["krylov_iterations"]}
        if oracle_u is not None:
            entry["state_rel_l2_vs_oracle"] = _rel(u.cpu().numpy(), oracle_u)
        out[name] = entry
        log(f"{name}: {sec * 1e3:.1f} ms ({dof_steps / sec:.3e} DoF*steps/s) {entry}")
    return out


# HBM bytes per unknown of one streaming Krylov iteration (FP64 vectors in
# HBM, every sweep counted once; neighbour reads served by the caches; each
# preconditioner application reads r and five factor vectors and writes z)
STREAM_BYTES_PER_ITERATION = {"cg": 152, "bicgstab": 296}


def copy_bandwidth(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (GB/s, read + write bytes) of a
    plain 1 GiB copy: the practical HBM ceiling the streaming solvers'
    algorithmic rate is also quoted against."""
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
    HBM: algorithmic bytes (sweeps x unknowns x Krylov iterations) over each
    solver's event-timed launches (a wide launch is a whole chain, its host
    polls included)."""
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
    bpi = STREAM_BYTES_PER_ITERATION[p["krylov"]]
    forms = {16: ("stream_kernel<drift, BiCGStab>: one 1,024-thread work-group per task"),
             4: ("wide solver: many work-groups per task, one launch per Krylov phase for "
                 "all tasks of a launch (every streaming launch by default)")}
    roof = {}
    for c in st["shapes"]:
        if c["K"] != 0 or c["W"] not in forms:
            continue
        achieved = c["work"] * bpi / (c["ms"] / 1e3) / 1e9 if c["ms"] > 0 else None
        roof["one_group_per_task" if c["W"] == 16 else "wide"] = {
            "kernel": forms[c["W"]], "bound": "hbm", "achieved": achieved,
            "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS if achieved else None,
            "bytes_per_unknown_iteration": bpi, "ms": c["ms"],
            "krylov_work": c["work"], "launches": c["launches"]}
    if not roof:
        return None
    copy_gbps = copy_bandwidth(torch)
    for r in roof.values():
        r["copy_GBps"] = copy_gbps
        r["frac_of_copy"] = r["achieved"] / copy_gbps if r["achieved"] else None
    return {
        "workload": f"fp_osc2d at L = 14, L0 = 6: {plan.G} grids, {plan.slen} DoF per level, "
                    f"{p['nsteps']} steps, 2-level MGRIT c = 2, BiCGStab, FP64, Krylov 1e-10, "
                    f"coarse levels 1e-3, MGRIT 1e-9",
        "seconds": sec,
        "value": plan.slen * p["nsteps"] / sec,
        "mgrit_iterations": st["mgrit_iterations"],
        "krylov_iterations": st["krylov_iterations"],
        "roofline": roof,
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


if __name__ == "__main__":
    sys.exit(main())
