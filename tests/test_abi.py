"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point include/ctm.h declares, the ctypes mirror of ctm_problem has
the C layout, and invalid problems are rejected before any device work."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctm.h")

ctm = pytest.importorskip("paper_2509_22156_amd.ctm")
from workloads import make  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctm_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(ctm.lib(), n), n
    out = subprocess.run(["nm", "-D", "--defined-only", ctm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for n in names:
        assert n in exported, n
    assert sorted(ctm.exported_symbols()) == names


def test_problem_struct_layout_matches_c(tmp_path):
    fields = [f for f, _ in ctm.Problem._fields_]
    src = tmp_path / "layout.c"
    body = "\n".join(f'  printf("{f} %zu\\n", offsetof(ctm_problem, {f}));' for f in fields)
    src.write_text(f"""#include <stdio.h>
#include <stddef.h>
#include "ctm.h"
int main(void) {{
  printf("size %zu\\n", sizeof(ctm_problem));
  printf("stats %zu\\n", sizeof(ctm_stats));
  printf("tune %zu\\n", sizeof(ctm_tune_report));
{body}
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                        text=True, check=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(ctm.Problem)
    assert int(out["stats"]) == ctypes.sizeof(ctm.Stats)
    assert int(out["tune"]) == ctypes.sizeof(ctm.TuneReport)
    for f in fields:
        assert int(out[f]) == getattr(ctm.Problem, f).offset, f


def _create(prob):
    s, keep = ctm.problem_struct(prob)
    return s, keep


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: setattr(s, "d", 0), "d must be"),
    (lambda s: setattr(s, "d", 9), "d must be"),
    (lambda s: setattr(s, "level_min", 0), "level_min"),
    (lambda s: setattr(s, "level_min", 5), "no component grid"),
    (lambda s: setattr(s, "nsteps", 63), "divisible"),
    (lambda s: setattr(s, "nrecomb", 5), "nrecomb"),
    (lambda s: setattr(s, "mgrit_cf", 1), "mgrit_cf"),
    (lambda s: setattr(s, "krylov_tol", 0.0), "krylov_tol"),
    (lambda s: setattr(s, "mgrit_tol", -1.0), "mgrit_tol"),
    (lambda s: setattr(s, "ic_terms", 0), "initial value"),
    (lambda s: setattr(s, "t1", -1.0), "t1"),
    (lambda s: setattr(s, "coarse_tol", -1e-3), "coarse_tol"),
    (lambda s: setattr(s, "coarse_tol", 1.0), "coarse_tol"),
    (lambda s: (setattr(s, "residual_mode", 1), setattr(s, "manufactured", 1)), "residual_mode"),
    (lambda s: (setattr(s, "residual_mode", 1), setattr(s, "mgrit_levels", 1)), "residual_mode"),
    (lambda s: (setattr(s, "residual_mode", 1), setattr(s, "warm_start", 0)), "residual_mode"),
    (lambda s: setattr(s, "residual_mode", 2), "residual_mode"),
])
def test_invalid_problems_rejected_on_host(mutate, msg):
    s, keep = _create(make("heat2d"))
    mutate(s)
    h = ctypes.c_void_p()
    st = ctm.lib().ctm_plan_create(ctypes.byref(s), ctypes.byref(h))
    assert st == ctm.ERR_INVALID
    assert msg in ctm.lib().ctm_last_error().decode()
    assert not h.value


def test_cg_rejected_for_nonsymmetric_and_lattice_box():
    s, keep = _create(make("ou4d"))
    s.krylov = 1
    h = ctypes.c_void_p()
    assert ctm.lib().ctm_plan_create(ctypes.byref(s), ctypes.byref(h)) == ctm.ERR_INVALID
    s, keep = _create(make("cme5d"))
    s.hi[0] = 60.0
    assert ctm.lib().ctm_plan_create(ctypes.byref(s), ctypes.byref(h)) == ctm.ERR_INVALID
    assert "2^n" in ctm.lib().ctm_last_error().decode()


def test_status_strings():
    for st in range(7):
        assert ctm.lib().ctm_status_string(st)


def test_long_lines_pass_validation():
    # lines of 2,047 unknowns (longer than one wave's 1,024-unknown line
    # segment) are accepted: the streaming preconditioner cuts them into
    # segments. Without a GPU the plan stops at its first device allocation
    # (a HIP error, not a validation error); with one it is built.
    s, keep = ctm.problem_struct(make("heat2d", n=12))
    h = ctypes.c_void_p()
    st = ctm.lib().ctm_plan_create(ctypes.byref(s), ctypes.byref(h))
    assert st in (ctm.OK, ctm.ERR_HIP), ctm.lib().ctm_last_error().decode()
    if st == ctm.OK:
        ctm.lib().ctm_plan_destroy(h)
    else:
        assert "longer" not in ctm.lib().ctm_last_error().decode()
        assert not h.value


def test_shape_entry_points_reject_null_plan():
    lib = ctm.lib()
    w, k = ctypes.c_int(), ctypes.c_int()
    assert lib.ctm_plan_grid_shape(None, 0, ctypes.byref(w), ctypes.byref(k)) == 1
    assert lib.ctm_plan_set_grid_shape(None, 0, 1, 4) == 1
    assert lib.ctm_plan_set_wide(None, 4) == 1
    assert lib.ctm_plan_set_schedule(None, ctm.SCHED_JOINED) == 1
    rep = ctm.TuneReport()
    assert lib.ctm_autotune(None, None, 0, None, 0, 1, ctypes.byref(rep), None) == 1
    assert "NULL" in lib.ctm_last_error().decode()


def test_stats_struct_layout_matches_c(tmp_path):
    fields = [f for f, _ in ctm.Stats._fields_]
    src = tmp_path / "stats.c"
    body = "\n".join(f'  printf("{f} %zu\\n", offsetof(ctm_stats, {f}));' for f in fields)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "ctm.h"\n'
                   f'int main(void) {{\n{body}\n  printf("size %zu\\n", sizeof(ctm_stats));\n'
                   f'  return 0;\n}}\n')
    exe = tmp_path / "stats"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.splitlines())
    for f in fields:
        assert int(got[f]) == getattr(ctm.Stats, f).offset, f
    assert int(got["size"]) == ctypes.sizeof(ctm.Stats)


@pytest.mark.parametrize("make_bad,err", [
    (lambda torch: [0.0] * 8, TypeError),
    (lambda torch: torch.zeros(8, dtype=torch.float32), TypeError),
    (lambda torch: torch.zeros(8, dtype=torch.float64), ValueError),          # host memory
])
def test_device_vector_guard_rejects_bad_inputs(make_bad, err):
    # every tensor handed to the library goes through this guard before its
    # raw pointer reaches a kernel; on the host the checks run up to the
    # device test
    import torch
    with pytest.raises(err):
        ctm._device_vec(make_bad(torch), 8, "x")
