"""Contraction paths and slicing choices (the upstream inputs of the method).

The paper takes its path from an external path finder; none is available
here, so these stand-ins produce the paths the benchmarks use:

``greedy_path``  repeatedly contracts the pair of tensors sharing at least one
    non-batch label whose result is smallest; ties go to the smaller
    size(out) - size(a) - size(b), then to the lower SSA ids.  Pieces left
    disconnected are joined by outer products, smallest first.
``random_greedy_path``  the same with the size key perturbed by seeded noise:
    a different, valid path used to show order independence.
``greedy_slice``  picks labels to slice one at a time, each the label of the
    currently largest tensor whose slicing gives the smallest largest tensor,
    ties to fewer total operations, then to the lower label.

A batch label (open and carried by two or more leaves) is never contracted;
sizes count it like any other mode.
"""
from __future__ import annotations

import heapq
import math
from typing import Dict, Iterable, List, Optional, Sequence, Set, Tuple

import numpy as np

from .network import Network, Path


def _size(labels: Iterable[int], ext: np.ndarray) -> int:
    s = 1
    for l in labels:
        s *= int(ext[l])
    return s


def _batch_labels(net: Network) -> Set[int]:
    cnt: Dict[int, int] = {}
    for lab in net.labels:
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    return {l for l in net.open if cnt.get(l, 0) >= 2}


def _out_labels(la: frozenset, lb: frozenset, keep: Set[int]) -> frozenset:
    """Labels of the result of contracting two tensors: shared labels are
    summed unless they must be kept (open labels, batch labels, or labels
    still held by some other tensor)."""
    shared = la & lb
    return (la | lb) - (shared - keep)


def _run_greedy(net: Network, noise: Optional[np.random.Generator], temperature: float,
                removed: Sequence[int] = ()) -> np.ndarray:
    ext = net.extents
    rem = set(removed)
    batch = _batch_labels(net)
    open_set = set(net.open)
    tens: Dict[int, frozenset] = {t: frozenset(l for l in lab if l not in rem)
                                  for t, lab in enumerate(net.labels)}
    owners: Dict[int, Set[int]] = {}
    for t, lab in tens.items():
        for l in lab:
            owners.setdefault(l, set()).add(t)
    size = {t: _size(lab, ext) for t, lab in tens.items()}
    heap: List[tuple] = []

    def keep_set(a: int, b: int) -> Set[int]:
        ks = set(open_set)
        for l in tens[a] & tens[b]:
            if len(owners[l]) > 2:
                ks.add(l)
        return ks

    def push(a: int, b: int) -> None:
        if a > b:
            a, b = b, a
        out = _out_labels(tens[a], tens[b], keep_set(a, b))
        so = _size(out, ext)
        k1 = math.log2(so)
        if noise is not None:
            k1 -= temperature * math.log(-math.log(noise.random() + 1e-300) + 1e-300)
        heapq.heappush(heap, (k1, so - size[a] - size[b], a, b))

    for l, ow in owners.items():
        if l in batch:
            continue
        ow = sorted(ow)
        for i in range(len(ow)):
            for j in range(i + 1, len(ow)):
                push(ow[i], ow[j])
    pairs = []
    nid = net.n_leaves
    alive = set(tens)
    while len(alive) > 1:
        pick = None
        while heap:
            _, _, a, b = heapq.heappop(heap)
            if a in alive and b in alive:
                pick = (a, b)
                break
        if pick is None:
            # disconnected pieces: outer product of the two smallest
            order = sorted(alive, key=lambda t: (size[t], t))
            pick = (order[0], order[1])
        a, b = pick
        out = _out_labels(tens[a], tens[b], keep_set(a, b))
        for t in (a, b):
            for l in tens[t]:
                owners[l].discard(t)
            alive.discard(t)
        tens[nid] = out
        size[nid] = _size(out, ext)
        for l in out:
            owners.setdefault(l, set()).add(nid)
        alive.add(nid)
        pairs.append((a, b))
        neigh = set()
        for l in out:
            if l in batch:
                continue
            neigh |= owners[l]
        neigh.discard(nid)
        for t in sorted(neigh):
            push(t, nid)
        nid += 1
    return np.array(pairs, dtype=np.int32).reshape(-1, 2)


def greedy_path(net: Network, sliced: Sequence[int] = ()) -> Path:
    return Path(_run_greedy(net, None, 0.0, sliced), tuple(sliced))


def random_greedy_path(net: Network, seed: int, temperature: float = 1.0) -> Path:
    rng = np.random.Generator(np.random.PCG64(seed))
    return Path(_run_greedy(net, rng, temperature), ())


def path_tensors(net: Network, pairs: np.ndarray, sliced: Sequence[int] = ()):
    """Label sets of every tensor (leaves then intermediates) along a path,
    with the sliced labels removed, and the per-step operation counts
    (product of the extents of all labels the step touches)."""
    ext = net.extents
    rem = set(sliced)
    open_set = set(net.open)
    cnt: Dict[int, int] = {}
    for lab in net.labels:
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    tens = [frozenset(l for l in lab if l not in rem) for lab in net.labels]
    live_cnt = dict(cnt)
    ops = []
    for a, b in pairs:
        la, lb = tens[a], tens[b]
        shared = la & lb
        keep = {l for l in shared if l in open_set or live_cnt[l] > 2}
        out = (la | lb) - (shared - keep)
        for l in shared - keep:
            live_cnt[l] -= 2
        for l in shared & keep:
            live_cnt[l] -= 1
        tens.append(out)
        ops.append(_size(la | lb, ext))
    return tens, ops


def path_cost(net: Network, pairs: np.ndarray, sliced: Sequence[int] = ()) -> Tuple[int, int]:
    """(largest tensor size, total operation count) of one slice."""
    tens, ops = path_tensors(net, pairs, sliced)
    return max(_size(t, net.extents) for t in tens), int(sum(ops))


def greedy_slice(net: Network, pairs: np.ndarray, n_sliced: Optional[int] = None,
                 max_size: Optional[int] = None) -> Tuple[int, ...]:
    """Choose labels to slice for a fixed path (see module doc)."""
    sliced: List[int] = []
    open_set = set(net.open)
    ext = net.extents
    while True:
        tens, _ = path_tensors(net, pairs, sliced)
        sizes = [_size(t, ext) for t in tens]
        big = int(np.argmax(sizes))
        if n_sliced is not None and len(sliced) >= n_sliced:
            break
        if max_size is not None and sizes[big] <= max_size and n_sliced is None:
            break
        cands = sorted(l for l in tens[big] if l not in open_set)
        if not cands:
            break
        best = None
        for l in cands:
            c = path_cost(net, pairs, sliced + [l])
            key = (c[0], c[1], l)
            if best is None or key < best:
                best = key
        sliced.append(best[2])
    return tuple(sliced)
