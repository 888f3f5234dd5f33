"""The plan and driver code of the library (csrc/ctm_host.cpp, and the
Schwarz decomposition of csrc/schwarz_plan.cpp) built for the
host with AddressSanitizer and UndefinedBehaviorSanitizer, linked with
launcher stubs instead of the device kernels (tests/asan/stubs.cpp), and
driven through the C ABI by tests/asan/driver.cpp: validation and rejection
of problems, enumeration, tables, launch shapes and scratch sizing of plan
creation for every operator, the shape entry points and destroy, and NULL
arguments everywhere. Any heap error, leak of the plan's host memory or
undefined behaviour aborts the driver.

On a host without a GPU plan creation stops at its first device allocation
and the error path releases the plan; the GPU-marked copy runs the same
driver where the allocations succeed, so every plan is built in full and
destroyed (the device is used for allocations only; no kernel runs)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# the host compiler builds the file's host side only: the two HIP spellings
# that only the HIP compiler knows get their host meaning
FLAGS = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-D__align__(n)=__attribute__((aligned(n)))",
         "-DHIP_SYMBOL(x)=(&(x))", "-Wno-unused-result", "-g", "-O1",
         "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-I", os.path.join(ROCM, "include"),
         "-I", os.path.join(ROOT, "include"),
         "-I", os.path.join(ROOT, "paper_2509_22156_amd", "csrc")]


def _build(tmp_path):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("needs g++ and the HIP runtime library")
    exe = tmp_path / "host_driver"
    srcs = [os.path.join(ROOT, "paper_2509_22156_amd", "csrc", "ctm_host.cpp"),
            os.path.join(ROOT, "paper_2509_22156_amd", "csrc", "schwarz_plan.cpp"),
            os.path.join(ROOT, "tests", "asan", "stubs.cpp"),
            os.path.join(ROOT, "tests", "asan", "driver.cpp")]
    objs = []
    for src in srcs:
        obj = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run(["g++", *FLAGS, "-c", src, "-o", str(obj)], check=True,
                       capture_output=True, text=True)
        objs.append(str(obj))
    subprocess.run(["g++", "-fsanitize=address,undefined", *objs, "-L",
                    os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    return exe


def _run(exe):
    supp = os.path.join(ROOT, "tests", "asan", "lsan.supp")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "all host checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_host_code_under_sanitizers(tmp_path):
    _run(_build(tmp_path))


@pytest.mark.gpu
def test_host_code_under_sanitizers_with_device_allocations(tmp_path):
    _run(_build(tmp_path))
