"""Containers for a tensor network, a contraction path, and their file format.

A network is a list of leaf tensors.  Leaf ``t`` has modes ``labels[t]``
(mode 0 outermost, row-major storage) and every label ``l`` has one extent
``extents[l]``.  A closed label joins exactly two leaves and is summed over;
an open label survives into the result, whose mode order is ``open``.  An
open label carried by two or more leaves is a batch label: it is kept, not
summed, wherever it meets (an independent problem per value).

A path is a list of SSA pairs: ids below ``n_leaves`` are leaves and step
``s`` creates id ``n_leaves + s``.  ``sliced`` lists closed labels whose
values are fixed per slice; the result is the sum over all slices, slice
index row-major over ``sliced`` (first label most significant).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Network:
    leaves: List[np.ndarray]            # complex128 (generated) or complex64
    labels: List[Tuple[int, ...]]       # per leaf, mode order of its storage
    extents: np.ndarray                 # int64, indexed by label
    open: Tuple[int, ...] = ()          # result mode order

    @property
    def n_leaves(self) -> int:
        return len(self.leaves)

    @property
    def n_labels(self) -> int:
        return int(len(self.extents))

    def c64(self) -> "Network":
        """The same network with complex64 leaves (the values both sides use)."""
        return Network([np.ascontiguousarray(x, dtype=np.complex64) for x in self.leaves],
                       list(self.labels), self.extents.copy(), tuple(self.open))

    def check_shapes(self) -> None:
        for t, (x, lab) in enumerate(zip(self.leaves, self.labels)):
            want = tuple(int(self.extents[l]) for l in lab)
            if tuple(x.shape) != want:
                raise ValueError(f"leaf {t}: shape {x.shape} != extents {want}")


@dataclasses.dataclass
class Path:
    pairs: np.ndarray                   # int32 [n_steps, 2], SSA ids
    sliced: Tuple[int, ...] = ()

    @property
    def n_steps(self) -> int:
        return int(self.pairs.shape[0])

    def n_slices(self, extents: np.ndarray) -> int:
        n = 1
        for l in self.sliced:
            n *= int(extents[l])
        return n


def save_tnz(path: str, net: Network, p: Path | None = None) -> None:
    """Write network (+ optional path) to an npz file (no pickled objects)."""
    ranks = np.array([len(l) for l in net.labels], dtype=np.int32)
    flat = np.array([x for l in net.labels for x in l], dtype=np.int32)
    data = {f"leaf{t}": np.ascontiguousarray(x) for t, x in enumerate(net.leaves)}
    data.update(ranks=ranks, labels=flat, extents=net.extents.astype(np.int64),
                open=np.array(net.open, dtype=np.int32))
    if p is not None:
        data.update(pairs=p.pairs.astype(np.int32), sliced=np.array(p.sliced, dtype=np.int32))
    np.savez(path, **data)


def load_tnz(path: str) -> Tuple[Network, Path | None]:
    z = np.load(path, allow_pickle=False)
    ranks = z["ranks"]
    flat = z["labels"]
    labels, pos = [], 0
    for r in ranks:
        labels.append(tuple(int(v) for v in flat[pos:pos + r]))
        pos += int(r)
    leaves = [z[f"leaf{t}"] for t in range(len(ranks))]
    net = Network(leaves, labels, z["extents"].astype(np.int64), tuple(int(v) for v in z["open"]))
    p = None
    if "pairs" in z:
        p = Path(z["pairs"].astype(np.int32), tuple(int(v) for v in z["sliced"]))
    return net, p


def flat_labels(labels: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    ranks = np.array([len(l) for l in labels], dtype=np.int32)
    flat = np.array([x for l in labels for x in l], dtype=np.int32)
    return ranks, flat
