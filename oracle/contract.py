"""Exact FP64 contraction of a tensor network along a pairwise path.

ORACLE -- test infrastructure only (see the package header).

Definition followed (paper Sec. II-A and II-B): a network is a set of
tensors joined by shared labels; a closed label joins two tensors and is
summed over, an open label survives into the result.  A contraction path is
an ordered sequence of pairwise contractions; each pairwise step sums the
labels its two operands share (C_ij = sum_k A_ik B_kj generalised to many
modes).  The result does not depend on the path.  Slicing (Sec. II-C) fixes
chosen closed labels to each of their values, contracts every such
sub-network independently and sums the partial results.

An open label carried by two or more leaves (a batch label) is kept where
two operands share it: each of its values is an independent problem.

Every step here is a plain ``numpy.tensordot`` in complex128; nothing is
blocked, fused or reordered.  Leaf values are taken as given (callers pass
the complex64 values upcast to complex128).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def label_kinds(labels: Sequence[Sequence[int]], open_labels: Sequence[int]) -> Dict[int, str]:
    """Classify each label as 'closed', 'open' or 'batch'; raise on anything
    that is not a tensor network in the paper's sense (a closed label must
    join exactly two tensors)."""
    cnt: Dict[int, int] = {}
    for t, lab in enumerate(labels):
        if len(set(lab)) != len(lab):
            raise ValueError(f"leaf {t} repeats a label")
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    op = list(open_labels)
    if len(set(op)) != len(op):
        raise ValueError("open list repeats a label")
    kinds = {}
    for l, c in cnt.items():
        if l in op:
            kinds[l] = "open" if c == 1 else "batch"
        elif c == 2:
            kinds[l] = "closed"
        else:
            raise ValueError(f"closed label {l} is held by {c} tensors (must be 2)")
    for l in op:
        if l not in cnt:
            raise ValueError(f"open label {l} is on no tensor")
    return kinds


def check_path(n_leaves: int, pairs: np.ndarray) -> None:
    """A path must consume every id exactly once and build one binary tree."""
    used = set()
    n_ids = n_leaves
    for a, b in np.asarray(pairs).reshape(-1, 2):
        a, b = int(a), int(b)
        if a == b or not (0 <= a < n_ids) or not (0 <= b < n_ids) or a in used or b in used:
            raise ValueError(f"invalid path pair ({a}, {b})")
        used.update((a, b))
        n_ids += 1
    if n_ids - n_leaves != max(n_leaves - 1, 0):
        raise ValueError("path does not join all leaves into one tree")


def pairwise(x: np.ndarray, la: List[int], y: np.ndarray, lb: List[int],
             keep: set) -> Tuple[np.ndarray, List[int]]:
    """Contract two tensors: sum the shared labels not in ``keep``.

    Result modes: kept shared labels, then x's other labels, then y's."""
    shared = [l for l in la if l in lb]
    summed = [l for l in shared if l not in keep]
    kept = [l for l in shared if l in keep]
    ra = [l for l in la if l not in shared]
    rb = [l for l in lb if l not in shared]
    ax = [la.index(l) for l in summed]
    ay = [lb.index(l) for l in summed]
    if not kept:
        z = np.tensordot(x, y, axes=(ax, ay))
        return z, ra + rb
    # batch labels: one independent tensordot per value combination
    kx = [la.index(l) for l in kept]
    ky = [lb.index(l) for l in kept]
    ext = [x.shape[i] for i in kx]
    out = None
    for idx in itertools.product(*[range(e) for e in ext]):
        sx = [slice(None)] * x.ndim
        sy = [slice(None)] * y.ndim
        for i, v in zip(kx, idx):
            sx[i] = v
        for i, v in zip(ky, idx):
            sy[i] = v
        xs, ys = x[tuple(sx)], y[tuple(sy)]
        la2 = [l for l in la if l not in kept]
        lb2 = [l for l in lb if l not in kept]
        z = np.tensordot(xs, ys, axes=([la2.index(l) for l in summed], [lb2.index(l) for l in summed]))
        if out is None:
            out = np.empty(tuple(ext) + z.shape, dtype=z.dtype)
        out[idx] = z
    return out, kept + ra + rb


def contract_tree(leaves: Sequence[np.ndarray], labels: Sequence[Sequence[int]],
                  open_labels: Sequence[int], pairs: np.ndarray, step=None) -> np.ndarray:
    """Contract along the SSA path; return the result in ``open_labels`` order.

    ``step(x, la, y, lb, keep)`` may replace the pairwise product (used by the
    split-precision emulation); it defaults to :func:`pairwise`."""
    step = step or pairwise
    open_set = set(open_labels)
    cnt: Dict[int, int] = {}
    for lab in labels:
        for l in lab:
            cnt[l] = cnt.get(l, 0) + 1
    tens: List[Optional[np.ndarray]] = [np.asarray(x) for x in leaves]
    labs: List[Optional[List[int]]] = [list(l) for l in labels]
    for a, b in np.asarray(pairs).reshape(-1, 2):
        a, b = int(a), int(b)
        la, lb = labs[a], labs[b]
        shared = [l for l in la if l in lb]
        keep = {l for l in shared if l in open_set or cnt[l] > 2}
        z, lz = step(tens[a], la, tens[b], lb, keep)
        for l in shared:
            cnt[l] -= 1 if l in keep else 2
        tens[a] = tens[b] = None
        labs[a] = labs[b] = None
        tens.append(z)
        labs.append(lz)
    root, lr = tens[-1], labs[-1]
    if len(leaves) == 1:
        root, lr = tens[0], labs[0]
    if sorted(lr) != sorted(open_labels):
        raise ValueError(f"root labels {lr} != open labels {list(open_labels)}")
    return np.transpose(root, [lr.index(l) for l in open_labels])


def slice_values(extents: np.ndarray, sliced: Sequence[int], s: int) -> Dict[int, int]:
    """Values of the sliced labels for slice s (row-major, first most significant)."""
    vals = {}
    for l in reversed(list(sliced)):
        d = int(extents[l])
        vals[l] = s % d
        s //= d
    return vals


def fix_labels(x: np.ndarray, lab: Sequence[int], vals: Dict[int, int]) -> Tuple[np.ndarray, List[int]]:
    idx = tuple(vals[l] if l in vals else slice(None) for l in lab)
    return x[idx], [l for l in lab if l not in vals]


def contract(net, path, slices: Optional[Sequence[int]] = None, step=None,
             leaves: Optional[Sequence[np.ndarray]] = None) -> np.ndarray:
    """Sum over slices (all by default) of the sliced sub-network contractions.

    ``leaves`` defaults to the network's complex64 values upcast to complex128.
    Partial results are added in the order given (slice order by default)."""
    label_kinds(net.labels, net.open)
    check_path(net.n_leaves, path.pairs)
    if leaves is None:
        leaves = [np.asarray(x, dtype=np.complex64).astype(np.complex128) for x in net.leaves]
    sliced = list(path.sliced)
    for l in sliced:
        if l in net.open:
            raise ValueError("open labels cannot be sliced")
    n_sl = path.n_slices(net.extents)
    todo = range(n_sl) if slices is None else slices
    acc = None
    for s in todo:
        vals = slice_values(net.extents, sliced, int(s))
        fl, fb = [], []
        for x, lab in zip(leaves, net.labels):
            y, l2 = fix_labels(x, lab, vals)
            fl.append(y)
            fb.append(l2)
        r = contract_tree(fl, fb, net.open, path.pairs, step=step)
        acc = r.astype(np.complex128) if acc is None else acc + r
    return acc
