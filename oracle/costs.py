"""Per-step GEMM sizes and path costs (paper Sec. II-B, Eq. (1)-(3)).

ORACLE -- test infrastructure only (see the package header).

For a pairwise step A_MK x B_KN -> C_MN with m, n, k the products of the
extents of the retained (M, N) and reduced (K) labels:
    C_t = m n k,   C_s = max(mk, kn, mn),   C_m = mk + kn + mn,
path totals C_t = sum C_t^(a), C_m = sum C_m^(a), C_s = max C_s^(a).
A batch group H (labels kept by both operands) multiplies every term by h,
the product of its extents, where an operand lacking a batch label counts it
once.  Complex arithmetic: one complex multiply-add = 8 real FLOPs.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np


def prod(ls, ext) -> int:
    p = 1
    for l in ls:
        p *= int(ext[l])
    return p


def step_costs(steps: List[dict], target: List[List[int]], extents: np.ndarray) -> List[Dict[str, int]]:
    """Costs of each step given the groups from the reordering pass."""
    out = []
    for st in steps:
        h = prod(st["H"], extents)
        m = prod(st["M"], extents)
        n = prod(st["N"], extents)
        k = prod(st["K"], extents)
        ha = prod([l for l in st["H"] if l in target[st["A"]]], extents)
        hb = prod([l for l in st["H"] if l in target[st["B"]]], extents)
        out.append(dict(h=h, m=m, n=n, k=k,
                        Ct=h * m * n * k,
                        Cs=max(ha * m * k, hb * k * n, h * m * n),
                        Cm=ha * m * k + hb * k * n + h * m * n))
    return out


def path_totals(costs: List[Dict[str, int]]) -> Dict[str, int]:
    return dict(Ct=sum(c["Ct"] for c in costs),
                Cm=sum(c["Cm"] for c in costs),
                Cs=max(c["Cs"] for c in costs) if costs else 0,
                flops=8 * sum(c["Ct"] for c in costs))
