"""Pins of the oracle's combination index set against numbers the paper prints."""
import os
from math import comb

import pytest

from oracle import index_set

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    with open(os.path.join(GOLD, "table1_process_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("d,L,P", _table1())
def test_table1_process_counts(d, L, P):
    # Section 4.2, Table 1: P = sum over all subproblems of ceil(|Omega_l| / 2^10)
    grids = index_set.combination_grids(d, L, 1)
    assert sum(index_set.spatial_processes(l, 10) for (l, _, _) in grids) == P


def _experiments():
    rows = []
    with open(os.path.join(GOLD, "experiment_subproblems.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, d, L, L0, S, tf, total, ms = line.split()
                rows.append((name, int(d), int(L), int(L0), int(S), int(tf), int(total),
                             sorted(int(v) for v in ms.split(","))))
    return rows


@pytest.mark.parametrize("name,d,L,L0,S,tf,total,procs", _experiments())
def test_experiment_subproblem_counts(name, d, L, L0, S, tf, total, procs):
    grids = index_set.combination_grids(d, L, L0)
    got = sorted(index_set.spatial_processes(l, S) for (l, _, _) in grids)
    assert got == procs
    assert tf * sum(got) == total


def test_single_grid_examples():
    # Section 2.1.2: l = (1, 11) has 2047 nodes and uses 2 processes at S = 10;
    # l = (6, 6) has 63^2 = 3969 nodes and uses 4.
    assert index_set.interior_points((1, 11)) == 2047
    assert index_set.interior_points((6, 6)) == 3969
    assert index_set.spatial_processes((1, 11), 10) == 2
    assert index_set.spatial_processes((6, 6), 10) == 4


def test_oscillator_dof_close_to_full_grid():
    # Section 4.4.1: the 421 x 421 full grid has approximately as many unknowns
    # as all subproblems of L = 14, L0 = 6 together.
    total = sum(index_set.interior_points(l) for (l, _, _) in index_set.combination_grids(2, 14, 6))
    assert total == 177415
    assert abs(total - 421 ** 2) / 421 ** 2 < 1e-3


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("L0", [1, 2])
def test_coefficients_sum_to_one(d, L0):
    for n in range(d * (L0 - 1) + 1, d * (L0 - 1) + 9):
        grids = index_set.combination_grids(d, n, L0)
        assert sum(c for (_, _, c) in grids) == 1


@pytest.mark.parametrize("d,n", [(2, 6), (3, 9), (4, 8), (5, 6), (6, 8)])
def test_layer_sizes_and_order(d, n):
    grids = index_set.combination_grids(d, n, 1)
    for w in range(d):
        layer = [l for (l, ww, _) in grids if ww == w]
        # number of compositions of n+d-1-w into d positive parts
        assert len(layer) == comb(n + d - 2 - w, d - 1)
        assert layer == sorted(layer)
        assert all(sum(l) == n + d - 1 - w and min(l) >= 1 for l in layer)
    ws = [w for (_, w, _) in grids]
    assert ws == sorted(ws)
    for (_, w, c) in grids:
        assert c == (-1) ** w * comb(d - 1, w)
