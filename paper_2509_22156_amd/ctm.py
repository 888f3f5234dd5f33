"""Python binding of the C ABI in include/ctm.h (argument marshalling only).

Device buffers are torch tensors on the current HIP device (float64); the
stream is torch's current stream. Every computation runs in the HIP
library; if libctm.so is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libctm.so")

MAXD = 8
MAX_HISTORY = 256
NOALLOC_WORKSPACE_BYTES = 256 << 20  # CTM_NOALLOC_WORKSPACE_BYTES of ctm.h

OK, ERR_INVALID, ERR_NOMEM, ERR_HIP, ERR_NOCONV, ERR_BREAKDOWN, ERR_NONFINITE = range(7)
SCHED_AUTO, SCHED_JOINED, SCHED_PER_CLASS = range(3)
_OPS = {"heat": 0, "varcoef": 1, "ou": 2, "cme": 3, "drift": 4}
_KRYLOV = {"auto": 0, "cg": 1, "bicgstab": 2}
_PREC = {"fp64": 0, "mixed": 1}
_RELAX = {"F": 0, "FCF": 1}
_PRECOND = {"line": 0, "schwarz": 1}


class Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int), ("level_n", ctypes.c_int), ("level_min", ctypes.c_int),
        ("lo", ctypes.c_double * MAXD), ("hi", ctypes.c_double * MAXD),
        ("op", ctypes.c_int), ("amp", ctypes.c_double),
        ("theta", ctypes.c_double * MAXD), ("sigma", ctypes.c_double),
        ("k", ctypes.c_double * MAXD), ("gamma", ctypes.c_double * MAXD),
        ("t0", ctypes.c_double), ("t1", ctypes.c_double),
        ("nsteps", ctypes.c_longlong), ("nrecomb", ctypes.c_int),
        ("mgrit_levels", ctypes.c_int), ("mgrit_cf", ctypes.c_int), ("relax", ctypes.c_int),
        ("mgrit_tol", ctypes.c_double), ("mgrit_maxit", ctypes.c_int),
        ("krylov", ctypes.c_int), ("krylov_tol", ctypes.c_double), ("krylov_maxit", ctypes.c_int),
        ("prec", ctypes.c_int), ("refine_tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
        ("refine_maxit", ctypes.c_int), ("ic_terms", ctypes.c_int),
        ("ic_weight", ctypes.POINTER(ctypes.c_double)),
        ("ic_factor", ctypes.POINTER(ctypes.c_double)),
        ("coarse_tol", ctypes.c_double), ("warm_start", ctypes.c_int),
        ("manufactured", ctypes.c_int),
        ("drift", ctypes.c_double * (MAXD * MAXD)), ("diffusion", ctypes.c_double * MAXD),
        ("residual_mode", ctypes.c_int),
        ("precond", ctypes.c_int), ("schwarz_s", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int), ("mgrit_iterations", ctypes.c_int),
        ("history_len", ctypes.c_int),
        ("mgrit_residual", ctypes.c_double * MAX_HISTORY),
        ("phi_solves", ctypes.c_longlong), ("krylov_iterations", ctypes.c_longlong),
        ("krylov_max", ctypes.c_longlong), ("refine_sweeps", ctypes.c_longlong),
        ("refine_max", ctypes.c_longlong), ("status_flags", ctypes.c_int),
        ("krylov_work", ctypes.c_longlong), ("chain_launches", ctypes.c_longlong),
        ("chain_ms", ctypes.c_double), ("chain_bytes", ctypes.c_double),
        ("shape_w", ctypes.c_int * 16), ("shape_k", ctypes.c_int * 16),
        ("shape_ms", ctypes.c_double * 16), ("shape_launches", ctypes.c_longlong * 16),
        ("shape_work", ctypes.c_longlong * 16), ("shape_bytes", ctypes.c_double * 16),
        ("shape_dofsteps", ctypes.c_longlong * 16),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [("classes", ctypes.c_int), ("trials", ctypes.c_int), ("changed", ctypes.c_int),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double),
                ("tune_ms", ctypes.c_double), ("schedule", ctypes.c_int)]


class CtmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ctm status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2509_22156_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i, ll, dbl, sz = ctypes.c_int, ctypes.c_longlong, ctypes.c_double, ctypes.c_size_t
    sigs = {
        "ctm_problem_defaults": [ctypes.POINTER(Problem)],
        "ctm_plan_create": [ctypes.POINTER(Problem), ctypes.POINTER(P)],
        "ctm_plan_grids": [P, ctypes.POINTER(i)],
        "ctm_plan_grid_info": [P, i, ctypes.POINTER(i), ctypes.POINTER(dbl), ctypes.POINTER(ll),
                               ctypes.POINTER(ll)],
        "ctm_plan_state_len": [P, ctypes.POINTER(ll)],
        "ctm_plan_workspace_bytes": [P, ctypes.POINTER(sz)],
        "ctm_initial_state": [P, P, P],
        "ctm_apply": [P, i, P, P, P],
        "ctm_precond_apply": [P, i, P, P, P],
        "ctm_propagate": [P, i, ll, P, P, i, P],
        "ctm_solve": [P, P, sz, P, P, P],
        "ctm_solve_noalloc": [P, P, P, P],
        "ctm_gather": [P, P, P, ll, P, P],
        "ctm_combine_project": [P, P, P, P],
        "ctm_hierarchize": [P, P, P, i, P],
        "ctm_recombine": [P, P, P, P],
        "ctm_get_stats": [P, ctypes.POINTER(Stats)],
        "ctm_set_timing": [P, i],
        "ctm_plan_grid_shape": [P, i, ctypes.POINTER(i), ctypes.POINTER(i)],
        "ctm_plan_set_grid_shape": [P, i, i, i],
        "ctm_plan_set_wide": [P, i],
        "ctm_plan_set_schedule": [P, i],
        "ctm_autotune": [P, P, sz, P, i, i, ctypes.POINTER(TuneReport), P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ctm_plan_destroy.argtypes = [P]
    lib.ctm_plan_destroy.restype = None
    lib.ctm_status_string.argtypes = [ctypes.c_int]
    lib.ctm_status_string.restype = ctypes.c_char_p
    lib.ctm_last_error.argtypes = []
    lib.ctm_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def _check(st: int):
    if st != OK:
        raise CtmError(st, _lib.ctm_last_error().decode())


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _device_vec(t, n: int, name: str):
    """Guard of every device vector handed to the library: a contiguous
    float64 tensor on the current HIP device holding at least n entries
    (the kernels read and write n entries through its raw pointer)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {t.dtype}")
    if not t.is_cuda or t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name}: expected a tensor on the current GPU, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if t.numel() < n:
        raise ValueError(f"{name}: holds {t.numel()} entries, needs at least {n}")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def problem_struct(prob: dict):
    """ctm_problem from a problem dictionary (see workloads); returns the
    struct and the numpy arrays it points to (keep them alive)."""
    s = Problem()
    _check(_lib.ctm_problem_defaults(ctypes.byref(s)))
    d = int(prob["d"])
    s.d, s.level_n, s.level_min = d, int(prob["n"]), int(prob.get("L0", 1))
    for i in range(d):
        s.lo[i] = float(prob["lo"][i])
        s.hi[i] = float(prob["hi"][i])
    s.op = _OPS[prob["op"]]
    s.amp = float(prob.get("amp", 0.0))
    for i in range(d):
        s.theta[i] = float(prob.get("theta", [0.0] * d)[i])
        s.k[i] = float(prob.get("k", [0.0] * d)[i])
        s.gamma[i] = float(prob.get("gamma", [0.0] * d)[i])
    s.sigma = float(prob.get("sigma", 0.0))
    s.t0, s.t1 = float(prob["t0"]), float(prob["t1"])
    s.nsteps = int(prob["nsteps"])
    s.nrecomb = int(prob.get("nrecomb", 1))
    s.mgrit_levels = int(prob.get("mgrit_levels", 2))
    s.mgrit_cf = int(prob.get("cf", 2))
    s.relax = _RELAX[prob.get("relax", "FCF")]
    s.mgrit_tol = float(prob.get("mgrit_tol", 1e-8))
    s.mgrit_maxit = int(prob.get("mgrit_maxit", 100))
    s.krylov = _KRYLOV[prob.get("krylov", "auto")]
    s.krylov_tol = float(prob.get("krylov_tol", 1e-8))
    s.krylov_maxit = int(prob.get("krylov_maxit", 10000))
    s.prec = _PREC[prob.get("prec", "fp64")]
    s.refine_tol = float(prob.get("refine_tol", 1e-8))
    s.inner_tol = float(prob.get("inner_tol", 1e-5))
    s.refine_maxit = int(prob.get("refine_maxit", 10))
    s.coarse_tol = float(prob.get("coarse_tol", 0.0))
    s.warm_start = int(prob.get("warm_start", 1))
    s.manufactured = 1 if prob.get("manufactured") == "heat" else 0
    s.residual_mode = int(prob.get("residual_mode", 0))
    s.precond = _PRECOND[prob.get("precond", "line")]
    s.schwarz_s = int(prob.get("schwarz_s", 5))
    if prob["op"] == "drift":
        th = np.asarray(prob["drift"], dtype=np.float64)
        for i in range(d):
            s.diffusion[i] = float(prob["diffusion"][i])
            for j in range(d):
                s.drift[i * d + j] = float(th[i, j])
    w = np.ascontiguousarray(prob["ic_w"], dtype=np.float64)
    f = np.ascontiguousarray(prob["ic_f"], dtype=np.float64)
    s.ic_terms = int(w.shape[0])
    s.ic_weight = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s.ic_factor = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return s, (w, f)


class Plan:
    """A plan for one problem: the component grids, their tables on the
    device, and the entry points of ctm.h."""

    def __init__(self, prob: dict):
        self.prob = prob
        s, keep = problem_struct(prob)
        h = ctypes.c_void_p()
        _check(_lib.ctm_plan_create(ctypes.byref(s), ctypes.byref(h)))
        self._h = h
        G = ctypes.c_int()
        _check(_lib.ctm_plan_grids(h, ctypes.byref(G)))
        self.G = G.value
        n = ctypes.c_longlong()
        _check(_lib.ctm_plan_state_len(h, ctypes.byref(n)))
        self.slen = n.value
        b = ctypes.c_size_t()
        _check(_lib.ctm_plan_workspace_bytes(h, ctypes.byref(b)))
        self.workspace_bytes = b.value
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ctm_plan_destroy(h)
            self._h = None

    def grid_info(self, g: int):
        lev = (ctypes.c_int * MAXD)()
        coef = ctypes.c_double()
        off = ctypes.c_longlong()
        npts = ctypes.c_longlong()
        _check(_lib.ctm_plan_grid_info(self._h, g, lev, ctypes.byref(coef), ctypes.byref(off),
                                       ctypes.byref(npts)))
        return tuple(lev[: self.prob["d"]]), coef.value, off.value, npts.value

    def _vec(self, out=None):
        if out is None:
            out = torch.empty(self.slen, dtype=torch.float64, device="cuda")
        return _device_vec(out, self.slen, "out")

    def _inp(self, x, name: str):
        return _device_vec(x, self.slen, name)

    def initial_state(self, out=None):
        out = self._vec(out)
        _check(_lib.ctm_initial_state(self._h, _ptr(out), _stream()))
        return out

    def apply(self, x, level: int = 0, out=None):
        self._inp(x, "x")
        out = self._vec(out)
        _check(_lib.ctm_apply(self._h, level, _ptr(x), _ptr(out), _stream()))
        return out

    def precond_apply(self, x, level: int = 0, out=None):
        """y = C x with the plan's Schwarz preconditioner (ctm_precond_apply)."""
        self._inp(x, "x")
        out = self._vec(out)
        _check(_lib.ctm_precond_apply(self._h, level, _ptr(x), _ptr(out), _stream()))
        return out

    def propagate(self, x, nsteps: int, level: int = 0, per_grid: bool = False, out=None):
        self._inp(x, "x")
        out = self._vec(out)
        _check(_lib.ctm_propagate(self._h, level, nsteps, _ptr(x), _ptr(out), int(per_grid),
                                  _stream()))
        return out

    def workspace(self):
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device="cuda")
        return self._ws

    def solve(self, u0=None, out=None, check: bool = True):
        """The whole method; returns the packed component states at t1.
        With check=False returns (state, status) instead of raising."""
        if u0 is not None:
            self._inp(u0, "u0")
        out = self._vec(out)
        ws = self.workspace()
        st = _lib.ctm_solve(self._h, _ptr(ws), ws.numel(), _ptr(u0), _ptr(out), _stream())
        if check:
            _check(st)
            return out
        return out, st

    def solve_noalloc(self, u0=None, out=None, check: bool = True):
        """The whole method on the library's static workspace
        (ctm_solve_noalloc): no device allocation inside the call."""
        if u0 is not None:
            self._inp(u0, "u0")
        out = self._vec(out)
        st = _lib.ctm_solve_noalloc(self._h, _ptr(u0), _ptr(out), _stream())
        if check:
            _check(st)
            return out
        return out, st

    def gather(self, u, pts, out=None):
        self._inp(u, "u")
        if pts.dim() != 2 or pts.shape[1] != self.prob["d"]:
            raise ValueError(f"pts: expected shape (n, {self.prob['d']}), got {tuple(pts.shape)}")
        _device_vec(pts, pts.numel(), "pts")
        if out is None:
            out = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
        _device_vec(out, pts.shape[0], "out")
        _check(_lib.ctm_gather(self._h, _ptr(u), _ptr(pts), pts.shape[0], _ptr(out), _stream()))
        return out

    def combine_project(self, u, out=None):
        self._inp(u, "u")
        out = self._vec(out)
        _check(_lib.ctm_combine_project(self._h, _ptr(u), _ptr(out), _stream()))
        return out

    def hierarchize(self, u, out=None, inverse=False):
        self._inp(u, "u")
        out = self._vec(out)
        _check(_lib.ctm_hierarchize(self._h, _ptr(u), _ptr(out), int(bool(inverse)), _stream()))
        return out

    def recombine(self, u, out=None):
        self._inp(u, "u")
        out = self._vec(out)
        _check(_lib.ctm_recombine(self._h, _ptr(u), _ptr(out), _stream()))
        return out

    def stats(self) -> dict:
        st = Stats()
        _check(_lib.ctm_get_stats(self._h, ctypes.byref(st)))
        return dict(blocks=st.blocks, mgrit_iterations=st.mgrit_iterations,
                    mgrit_residual=list(st.mgrit_residual[: st.history_len]),
                    phi_solves=st.phi_solves, krylov_iterations=st.krylov_iterations,
                    krylov_max=st.krylov_max, refine_sweeps=st.refine_sweeps,
                    refine_max=st.refine_max, status_flags=st.status_flags,
                    krylov_work=st.krylov_work, chain_launches=st.chain_launches,
                    chain_ms=st.chain_ms, chain_bytes=st.chain_bytes,
                    shapes=[dict(W=st.shape_w[i], K=st.shape_k[i], ms=st.shape_ms[i],
                                 launches=st.shape_launches[i], work=st.shape_work[i],
                                 bytes=st.shape_bytes[i], dofsteps=st.shape_dofsteps[i])
                            for i in range(16) if st.shape_launches[i] or st.shape_work[i]])

    def grid_shape(self, g: int):
        """(waves per work-group, unknowns per lane) of grid g; (16, 0) for
        the streaming solver."""
        w, k = ctypes.c_int(), ctypes.c_int()
        _check(_lib.ctm_plan_grid_shape(self._h, g, ctypes.byref(w), ctypes.byref(k)))
        return w.value, k.value

    def set_grid_shape(self, g: int, waves: int, per_lane: int):
        _check(_lib.ctm_plan_set_grid_shape(self._h, g, waves, per_lane))

    def set_wide(self, max_tasks: int):
        """Streaming-solver launches of at most max_tasks tasks run on the wide
        (many work-groups per task) solver; 0 disables it (default: every launch)."""
        _check(_lib.ctm_plan_set_wide(self._h, max_tasks))

    def set_schedule(self, schedule: int):
        """MGRIT phase schedule: SCHED_AUTO, SCHED_JOINED or SCHED_PER_CLASS
        (ctm_plan_set_schedule)."""
        _check(_lib.ctm_plan_set_schedule(self._h, int(schedule)))

    def autotune(self, trial_iterations: int = 0, repeats: int = 2) -> dict:
        """Choose the launch shape of every anisotropy class and the MGRIT
        schedule by timed trial solves (ctm_autotune); returns its report."""
        ws = self.workspace()
        u = self._vec()
        rep = TuneReport()
        _check(_lib.ctm_autotune(self._h, _ptr(ws), ws.numel(), _ptr(u), trial_iterations,
                                 repeats, ctypes.byref(rep), _stream()))
        return {k: getattr(rep, k) for k, _ in TuneReport._fields_}

    def set_timing(self, on: bool = True):
        _check(_lib.ctm_set_timing(self._h, int(on)))


def exported_symbols():
    """Names of the entry points declared in include/ctm.h."""
    return ["ctm_problem_defaults", "ctm_plan_create", "ctm_plan_destroy", "ctm_plan_grids",
            "ctm_plan_grid_info", "ctm_plan_state_len", "ctm_plan_workspace_bytes",
            "ctm_initial_state", "ctm_apply", "ctm_precond_apply", "ctm_propagate", "ctm_solve", "ctm_solve_noalloc",
            "ctm_gather",
            "ctm_combine_project", "ctm_hierarchize", "ctm_recombine", "ctm_get_stats", "ctm_set_timing", "ctm_plan_grid_shape",
            "ctm_plan_set_grid_shape", "ctm_plan_set_wide", "ctm_plan_set_schedule", "ctm_autotune", "ctm_status_string",
            "ctm_last_error"]
