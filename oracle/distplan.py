"""Mode-distribution planning along a use-chain, by exhaustive enumeration.

ORACLE -- test infrastructure only (see the package header).

What it computes (paper Sec. IV-B): along a use-chain of L contractions,
every equation either keeps the distributed modes it inherits or
redistributes to a fresh prefix of its output's modes; the schedule of
minimum total cost is wanted.  The paper finds it by dynamic programming; the
plain definition is the minimum over all 2^(L-1) keep/redistribute choices,
which is what this module evaluates (small L only).

Cost model, as the paper states it:
  * distributed modes (Eq. (4)): the shortest prefix of the tensor's mode
    order whose extents multiply to at least P;
  * per-equation time (Eq. (5)): t = t_gemm + [redistribute] * t_comm;
  * t_gemm (Eq. (6)) = max(D_rw / B_dev, FLOPs / F_dev) with per-device
    bytes and FLOPs: the chain operand and the output split P ways, the other
    operand whole on every device; 8 bytes per complex64 element and 8 FLOPs
    per complex multiply-add;
  * t_comm (Eq. (7)) = |C| (P-1) / (P B_net) + n_blk * max(lambda, s_blk / B_net),
    s_blk = bytes of one contiguous block (the modes after the innermost
    old-or-new distributed mode), n_blk = blocks per device;
  * a distributed mode about to be summed at the next equation forces a
    redistribution; the chain ends with a gather (all-gather of the last
    output: |C| (P-1) / (P B_net)).

Each equation of a chain is a dict with
  order  -- mode labels of its output, in storage order
  ext    -- label -> extent
  a, b, c -- element counts of the chain operand, the other operand, the output
  ops    -- complex multiply-adds (h m n k)
  next_summed -- labels of this output summed by the next equation (empty at
                 the end of the chain)
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Optional, Sequence, Tuple


def prefix_modes(order: Sequence[int], ext: Dict[int, int], P: int) -> Tuple[int, ...]:
    out, prod = [], 1
    for l in order:
        if prod >= P:
            break
        out.append(l)
        prod *= ext[l]
    if prod < P:
        return tuple()          # the tensor cannot be split P ways
    return tuple(out)


def t_gemm(eq: dict, P: int, hw: dict) -> float:
    d_rw = 8.0 * (eq["a"] / P + eq["b"] + eq["c"] / P)
    flops = 8.0 * eq["ops"] / P
    return max(d_rw / hw["B_dev"], flops / hw["F_dev"])


def t_comm(eq: dict, P: int, hw: dict, old: Tuple[int, ...], new: Tuple[int, ...]) -> float:
    order = list(eq["order"])
    pos = [order.index(l) for l in set(old) | set(new)]
    inner = 1
    for l in order[max(pos) + 1:] if pos else order:
        inner *= eq["ext"][l]
    s_blk = 8.0 * inner
    n_blk = math.ceil(8.0 * eq["c"] / P / s_blk)
    return 8.0 * eq["c"] * (P - 1) / (P * hw["B_net"]) + n_blk * max(hw["lat"], s_blk / hw["B_net"])


def t_gather(eq: dict, P: int, hw: dict) -> float:
    return 8.0 * eq["c"] * (P - 1) / (P * hw["B_net"])


def evaluate(chain: List[dict], P: int, hw: dict, redist: Sequence[bool]) -> Optional[float]:
    """Total time of one schedule (redist[i] for equations 1..L-1), or None if
    it keeps a distributed mode that the next equation sums."""
    D = prefix_modes(chain[0]["order"], chain[0]["ext"], P)
    if not D:
        return None
    total = t_gemm(chain[0], P, hw)
    if set(D) & set(chain[0]["next_summed"]):
        return None
    for i in range(1, len(chain)):
        eq = chain[i]
        total += t_gemm(eq, P, hw)
        if redist[i - 1]:
            new = prefix_modes(eq["order"], eq["ext"], P)
            if not new:
                return None
            total += t_comm(eq, P, hw, D, new)
            D = new
        if set(D) & set(eq["next_summed"]):
            return None
    return total + t_gather(chain[-1], P, hw)


def brute_force(chain: List[dict], P: int, hw: dict):
    """Minimum over every keep/redistribute schedule; ties go to the schedule
    that redistributes later (keep preferred, compared from the front)."""
    best = None
    for bits in itertools.product((False, True), repeat=len(chain) - 1):
        c = evaluate(chain, P, hw, bits)
        if c is None:
            continue
        if best is None or c < best[0] - 1e-12 * max(1.0, abs(c)):
            best = (c, bits)
    return best


def use_chains(labels, pairs, open_labels, extents, large_bytes: float):
    """The use-chains of a path (Sec. IV-B): a step is large when an operand or
    its output holds at least large_bytes (8 bytes per element); a chain runs
    from a large step through its output's consumers (the tensor's
    descendants) and ends at the last large step on that way up; chains do
    not share steps.  Mode orders are the reordering pass's targets."""
    from .costs import step_costs
    from .reorder import reorder

    target, steps = reorder(labels, pairs, open_labels)
    ext = {l: int(extents[l]) for l in range(len(extents))}
    n = len(labels)
    size = [1] * (n + len(steps))
    for i, order in enumerate(target):
        for l in order:
            size[i] *= ext[l]
    costs = step_costs(steps, target, extents)
    consumer = {}
    for s, (a, b) in enumerate(pairs):
        consumer[int(a)] = s
        consumer[int(b)] = s

    def large(s):
        st = steps[s]
        return 8 * max(size[st["A"]], size[st["B"]], size[st["C"]]) >= large_bytes

    covered = set()
    chains = []
    for s0 in range(len(steps)):
        if s0 in covered or not large(s0):
            continue
        chain = []
        t = s0
        while t is not None and t not in covered:
            chain.append(t)
            t = consumer.get(steps[t]["C"])
        while chain and not large(chain[-1]):
            chain.pop()
        covered.update(chain)
        eqs = []
        for i, t in enumerate(chain):
            st = steps[t]
            if i == 0:
                main = st["A"] if size[st["A"]] >= size[st["B"]] else st["B"]
            else:
                main = steps[chain[i - 1]]["C"]
            other = st["B"] if main == st["A"] else st["A"]
            order = list(target[st["C"]])
            nxt = [l for l in steps[chain[i + 1]]["K"] if l in order] if i + 1 < len(chain) else []
            eqs.append(dict(step=t, order=order, ext=ext, a=size[main], b=size[other], c=size[st["C"]],
                            ops=costs[t]["Ct"], next_summed=nxt))
        chains.append(eqs)
    return chains
