"""The library's host decomposition for the Schwarz preconditioner
(csrc/schwarz_plan.cpp: Hilbert-curve order with virtual nodes, partition,
overlap, weights, coarse blocks; Section 2.1.2), built for the host and
compared index for index with the oracle's (oracle/schwarz.py), which is
pinned on its own. Integer work: bit-exact."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import schwarz
from workloads import make

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = ["-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2509_22156_amd", "csrc")]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    out = tmp_path_factory.mktemp("decompose") / "decompose"
    subprocess.run(["g++", *FLAGS, os.path.join(ROOT, "tests", "host", "decompose.cpp"),
                    os.path.join(ROOT, "paper_2509_22156_amd", "csrc", "schwarz_plan.cpp"),
                    "-o", str(out)], check=True, capture_output=True, text=True)
    return str(out)


def _run(exe, lattice, S, l):
    args = [exe, str(len(l)), "0" if lattice else "1", str(S), *[str(x) for x in l]]
    lines = subprocess.run(args, check=True, capture_output=True, text=True).stdout.splitlines()
    return lines


@pytest.mark.parametrize("lattice,S,l", [
    (False, 3, (2, 3)), (False, 4, (5, 3)), (False, 5, (6, 4)), (False, 2, (3, 3)),
    (False, 4, (3, 2, 4)), (False, 6, (4, 4, 3)), (False, 3, (2, 2, 2, 3)),
    (False, 5, (1, 1, 1, 1, 1, 7)), (False, 4, (7, 1)), (False, 5, (2, 2, 2, 2, 2, 2)),
    (True, 3, (3, 4)), (True, 4, (2, 3, 2)),
])
def test_host_decomposition_matches_oracle(exe, lattice, S, l):
    p = make("cme5d", d=len(l), n=max(l) + 1, hi=[2.0 ** (max(l) + 1)] * len(l)) if lattice \
        else make("heat2d", d=len(l), n=max(l) + 1)
    dec = schwarz.Decomposition(p, l, S)
    lines = _run(exe, lattice, S, l)
    assert lines[-1] == "pairs ok"
    order = [int(x) for x in lines[0].split()[1:]]
    assert order == [int(x) for x in dec.order]
    blocks = [int(x) for x in lines[1].split()[1:]]
    assert blocks == [a for a, _ in dec.blocks] + [dec.N]
    subs = [ln.split() for ln in lines[2:-1]]
    assert len(subs) == dec.P
    for (a, b), om, sub in zip(dec.extended, dec.omega, subs):
        n = int(sub[1])
        assert n == b - a
        assert float(sub[2]) == om
        assert [int(x) for x in sub[3:]] == [int(x) for x in dec.order[a:b]]
