"""The wide streaming solver's work-group placement (csrc/wide_map.h), the
same functions the kernels call, built for the host: a bijection of every
launch's blocks onto (block, task) pairs, each task of a group of eight on
one XCD of the dispatcher's round robin, and the per-XCD regrouping of line
blocks a bijection with consecutive virtual blocks per XCD. Integer work:
exact."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = ["-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
         "-I", os.path.join(ROOT, "paper_2509_22156_amd", "csrc")]


def test_wide_block_mapping(tmp_path):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    exe = tmp_path / "wide_map"
    subprocess.run(["g++", *FLAGS, os.path.join(ROOT, "tests", "host", "wide_map.cpp"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe), "70", "41", "600"], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
