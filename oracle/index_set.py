"""Combination index set (Section 2.1.1, combination formula; Section 2.2.2,
definition of layer(Omega_l)).

The sparse-grid solution of level n (the paper's L) in d dimensions is

    u^(c) = sum_{w=0}^{d-1} (-1)^w binom(d-1, w) sum_{|l|_1 = n+d-1-w, l >= L0} u_l .

The subproblem l belongs to layer w = n + d - 1 - |l|_1 and carries the
coefficient (-1)^w binom(d-1, w).

Canonical order (also the packed-state order of the GPU library, an
interface convention): w ascending, then l in lexicographic order.

Pinned by: tests/test_oracle_index_set.py -- the process counts of the
paper's Table 1 (Section 4.2), the subproblem and process counts quoted for
the toggle-switch and oscillator experiments (Sections 4.3.1, 4.3.2, 4.4.1),
the two single-grid examples of Section 2.1.2, and the identity
sum_l c_l = 1.
"""
from __future__ import annotations

from math import comb


def compositions(total: int, parts: int, minimum: int):
    """All tuples of `parts` integers >= minimum summing to `total`, in
    lexicographic order."""
    if parts == 1:
        if total >= minimum:
            yield (total,)
        return
    for first in range(minimum, total - minimum * (parts - 1) + 1):
        for rest in compositions(total - first, parts - 1, minimum):
            yield (first,) + rest


def combination_grids(d: int, n: int, L0: int = 1):
    """List of (l, w, coefficient) for the combination of level n."""
    out = []
    for w in range(d):
        total = n + d - 1 - w
        if total < d * L0:
            continue
        coef = (-1) ** w * comb(d - 1, w)
        for l in compositions(total, d, L0):
            out.append((l, w, coef))
    return out


def interior_points(l, lattice: bool = False) -> int:
    """Unknowns of Omega_l: prod (2^{l_i} - 1) interior nodes for Dirichlet
    grids (Section 2.1.2, example after the process-count formula); prod
    2^{l_i} lattice states for the master-equation embedding."""
    p = 1
    for li in l:
        p *= (2 ** li) if lattice else (2 ** li - 1)
    return p


def spatial_processes(l, S: int) -> int:
    """P^x_l = ceil(|Omega_l| / 2^S) (Section 2.1.2, subproblem-dependent
    process count)."""
    pts = interior_points(l)
    return -(-pts // (2 ** S))
