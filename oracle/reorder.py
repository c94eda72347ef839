"""GEMM-oriented mode reordering: the backward pass of paper Sec. IV-A.

ORACLE -- test infrastructure only (see the package header).

What the pass computes (Sec. IV-A, its backward pass; worked example in
Fig. 3):
  * the root's mode order is the requested result order (its open labels);
  * visiting the steps from the last to the first, each step's output order
    is already known; each operand's order becomes
        [its labels kept by the step, in the output's order || labels summed here]
  * an operand produced by an earlier step passes that order on to its
    producer, whose output is then written in it (one consumer per tensor in
    a tree, so no conflicts).

Readings where the paper leaves a choice open (the same readings the
executor uses):
  * summed labels go in ascending label id (this reproduces Fig. 3's
    ``bf`` and ``cd``);
  * batch labels (open labels shared by several leaves, and the labels of a
    slice batch) lead every tensor in one canonical order and are never
    summed;
  * the operand whose labels hold the output's innermost non-batch label is
    the N side (B) of the GEMM; otherwise, and when there is no such label,
    the first operand of the pair is the M side (A).

Returns the target mode order of every tensor id (leaves first) and, per
step, the GEMM groups H (batch), M, N, K and whether the output is stored in
natural [H | M | N] order.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np


def reorder(labels: Sequence[Sequence[int]], pairs: np.ndarray, open_labels: Sequence[int],
            batch_order: Sequence[int] = ()):
    n_leaves = len(labels)
    pairs = np.asarray(pairs).reshape(-1, 2)
    batch = list(batch_order)
    bset = set(batch)
    open_set = set(open_labels)
    cnt: Dict[int, int] = {}
    for lab in labels:
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    sets: List[set] = [set(l) for l in labels]
    summed_at: List[set] = []
    for a, b in pairs:
        la, lb = sets[a], sets[b]
        shared = la & lb
        keep = {l for l in shared if l in open_set or l in bset or cnt[l] > 2}
        for l in shared:
            cnt[l] -= 1 if l in keep else 2
        summed_at.append(shared - keep)
        sets.append((la | lb) - (shared - keep))
    n_ids = len(sets)
    target: List[List[int]] = [None] * n_ids
    root = n_ids - 1
    target[root] = [l for l in batch if l in sets[root]] + \
        [l for l in open_labels if l in sets[root] and l not in bset]
    steps = [None] * len(pairs)
    for s in range(len(pairs) - 1, -1, -1):
        a, b = int(pairs[s][0]), int(pairs[s][1])
        out = n_leaves + s
        tc = target[out]
        K = sorted(summed_at[s])
        nonbatch = [l for l in tc if l not in bset]
        if nonbatch and nonbatch[-1] in sets[a]:
            a, b = b, a
        for x in (a, b):
            target[x] = [l for l in tc if l in sets[x]] + K
        H = [l for l in tc if l in bset]
        M = [l for l in tc if l in sets[a] and l not in bset]
        N = [l for l in tc if l in sets[b] and l not in bset]
        steps[s] = dict(A=a, B=b, C=out, H=H, M=M, N=N, K=K, natural=(tc == H + M + N))
    return target, steps


def lifetimes(labels: Sequence[Sequence[int]], pairs: np.ndarray, open_labels: Sequence[int],
              batch_order: Sequence[int] = ()) -> Dict[int, float]:
    """Step index at which each label is summed (inf for labels never summed):
    the tag of Sec. IV-B's distributed-mode tracking, and the lifetime key of
    the ordering that the backward pass produces."""
    bset = set(batch_order)
    open_set = set(open_labels)
    cnt: Dict[int, int] = {}
    for lab in labels:
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    sets: List[set] = [set(l) for l in labels]
    tag = {l: float("inf") for l in cnt}
    for s, (a, b) in enumerate(np.asarray(pairs).reshape(-1, 2)):
        shared = sets[a] & sets[b]
        keep = {l for l in shared if l in open_set or l in bset or cnt[l] > 2}
        for l in shared:
            cnt[l] -= 1 if l in keep else 2
        for l in shared - keep:
            tag[l] = s
        sets.append((sets[a] | sets[b]) - (shared - keep))
    return tag
