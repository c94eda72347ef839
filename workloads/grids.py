"""Closed 2D random tensor networks on an rows x cols grid.

Synthetic stand-in for the many-body-dynamics lattices of the paper's
experiments (their networks are not used here).  One leaf per grid node
(row-major), one label per grid edge: horizontal edges first (row-major by
their left node), then vertical edges (row-major by their top node).  A
node's modes are its incident edges in the order up, left, right, down.
Entries are i.i.d. complex Gaussian with E|z|^2 = 1 (real and imaginary
parts N(0, 1/2)) times 1/sqrt(numel), drawn node by node from
Generator(PCG64(seed)).

``prescale_log2`` gives an exact power-of-two factor per leaf,
2**floor(degree/2), that keeps the products of a deep contraction away from
the bottom of the float32 exponent range; a caller that applies it divides
the result by 2**sum(prescale_log2).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .network import Network


def grid_edges(rows: int, cols: int):
    h = {}
    v = {}
    lab = 0
    for r in range(rows):
        for c in range(cols - 1):
            h[(r, c)] = lab
            lab += 1
    for r in range(rows - 1):
        for c in range(cols):
            v[(r, c)] = lab
            lab += 1
    return h, v, lab


def grid_labels(rows: int, cols: int) -> Tuple[List[Tuple[int, ...]], int]:
    h, v, n_lab = grid_edges(rows, cols)
    labels = []
    for r in range(rows):
        for c in range(cols):
            mine = []
            if r > 0:
                mine.append(v[(r - 1, c)])      # up
            if c > 0:
                mine.append(h[(r, c - 1)])      # left
            if c < cols - 1:
                mine.append(h[(r, c)])          # right
            if r < rows - 1:
                mine.append(v[(r, c)])          # down
            labels.append(tuple(mine))
    return labels, n_lab


def random_grid_network(rows: int, cols: int, bond: int, seed: int) -> Network:
    labels, n_lab = grid_labels(rows, cols)
    rng = np.random.Generator(np.random.PCG64(seed))
    leaves = []
    for lab in labels:
        shape = (bond,) * len(lab)
        numel = bond ** len(lab)
        z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
        leaves.append(z / np.sqrt(numel))
    return Network(leaves, labels, np.full(n_lab, bond, dtype=np.int64), ())


def constant_grid_network(rows: int, cols: int, bond: int) -> Network:
    """Every entry 1/sqrt(numel): the closed network contracts to exactly
    prod_e d_e * prod_t numel_t**-1/2 = 1 (each edge sums d_e equal terms and
    each leaf's numel is the product of its incident extents)."""
    labels, n_lab = grid_labels(rows, cols)
    leaves = []
    for lab in labels:
        numel = bond ** len(lab)
        leaves.append(np.full((bond,) * len(lab), 1.0 / np.sqrt(numel), dtype=np.complex128))
    return Network(leaves, labels, np.full(n_lab, bond, dtype=np.int64), ())


def product_grid_network(rows: int, cols: int, bond: int, seed: int):
    """Leaves that are outer products of one vector per incident edge.

    Returns (network, vecs) with vecs[(t, l)] the factor of leaf t along
    label l; a closed network of such leaves contracts to the product over
    edges of the bilinear (unconjugated) products of the two factors.
    """
    labels, n_lab = grid_labels(rows, cols)
    rng = np.random.Generator(np.random.PCG64(seed))
    vecs = {}
    leaves = []
    for t, lab in enumerate(labels):
        parts = []
        for l in lab:
            v = (rng.standard_normal(bond) + 1j * rng.standard_normal(bond)) / np.sqrt(2.0 * bond)
            vecs[(t, l)] = v
            parts.append(v)
        x = parts[0]
        for v in parts[1:]:
            x = np.multiply.outer(x, v)
        leaves.append(np.ascontiguousarray(x))
    return Network(leaves, labels, np.full(n_lab, bond, dtype=np.int64), ()), vecs


def prescale_log2(labels: List[Tuple[int, ...]]) -> np.ndarray:
    return np.array([len(l) // 2 for l in labels], dtype=np.int64)
