"""Haar-random grid circuits and their tensor networks.

Circuit recipe (synthetic stand-in for the random-circuit-sampling workloads
of the paper's experiments, whose circuit instances are not used here):
  * qubit q = r * cols + c on an rows x cols grid;
  * one cycle = a Haar-random 2x2 unitary on every qubit (q ascending), then
    Haar-random 4x4 two-qubit gates on one edge pattern, patterns cycling
    A, B, C, D by cycle index mod 4:
      A: horizontal edges with even left column, B: horizontal, odd left column,
      C: vertical edges with even top row,       D: vertical, odd top row;
    edges within a pattern in ascending (q1, q2) order;
  * all qubits start in |0>; depth d = d cycles, no trailing layer;
  * Haar sampling = QR of a complex Ginibre matrix with the phases of R's
    diagonal moved into Q (Mezzadri's method), complex128;
  * RNG: numpy Generator(PCG64(seed)); draws in gate order, then the
    bitstring (one integer in {0,1} per qubit).

Gate tensors: a 1q gate is U[out, in]; a 2q gate on (q1 < q2) is
G[o1, o2, i1, i2] = M[2*o1 + o2, 2*i1 + i2].  The statevector index has
qubit 0 as its most significant bit.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .network import Network


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    diag = np.diagonal(r)
    return q * (diag / np.abs(diag))[None, :]


def pattern_edges(rows: int, cols: int, pattern: str) -> List[Tuple[int, int]]:
    edges = []
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if pattern in "AB" and c + 1 < cols and (c % 2 == (0 if pattern == "A" else 1)):
                edges.append((q, q + 1))
            if pattern in "CD" and r + 1 < rows and (r % 2 == (0 if pattern == "C" else 1)):
                edges.append((q, q + cols))
    return sorted(edges)


@dataclasses.dataclass
class Circuit:
    n_qubits: int
    rows: int
    cols: int
    depth: int
    # gates in application order: (qubits tuple, unitary complex128)
    gates: List[Tuple[Tuple[int, ...], np.ndarray]]
    bitstring: np.ndarray


def random_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rows * cols
    gates: List[Tuple[Tuple[int, ...], np.ndarray]] = []
    for t in range(depth):
        for q in range(n):
            gates.append(((q,), haar_unitary(rng, 2)))
        for (q1, q2) in pattern_edges(rows, cols, "ABCD"[t % 4]):
            gates.append(((q1, q2), haar_unitary(rng, 4)))
    bits = rng.integers(0, 2, size=n).astype(np.int8)
    return Circuit(n, rows, cols, depth, gates, bits)


def circuit_network(circ: Circuit, bitstring: Optional[Sequence[int]] = None,
                    open_qubits: Sequence[int] = ()) -> Network:
    """Tensor network of <x| C |0...0>.

    Qubits in ``open_qubits`` get no projector; their final wire labels are the
    result's open modes (in the given qubit order).  The others are projected
    on ``bitstring`` (default: the circuit's own seeded bitstring).
    """
    bits = circ.bitstring if bitstring is None else np.asarray(bitstring)
    leaves: List[np.ndarray] = []
    labels: List[Tuple[int, ...]] = []
    next_label = 0
    cur = []
    for q in range(circ.n_qubits):
        leaves.append(np.array([1.0, 0.0], dtype=np.complex128))
        labels.append((next_label,))
        cur.append(next_label)
        next_label += 1
    for qs, u in circ.gates:
        if len(qs) == 1:
            (q,) = qs
            leaves.append(np.ascontiguousarray(u))
            labels.append((next_label, cur[q]))
            cur[q] = next_label
            next_label += 1
        else:
            q1, q2 = qs
            leaves.append(np.ascontiguousarray(u.reshape(2, 2, 2, 2)))
            labels.append((next_label, next_label + 1, cur[q1], cur[q2]))
            cur[q1], cur[q2] = next_label, next_label + 1
            next_label += 2
    open_set = set(open_qubits)
    for q in range(circ.n_qubits):
        if q in open_set:
            continue
        v = np.zeros(2, dtype=np.complex128)
        v[int(bits[q])] = 1.0
        leaves.append(v)
        labels.append((cur[q],))
    extents = np.full(next_label, 2, dtype=np.int64)
    return Network(leaves, labels, extents, tuple(cur[q] for q in open_qubits))


def circuit_network_batched(circ: Circuit, bitstrings: np.ndarray) -> Network:
    """Tensor network of the amplitudes <x_b| C |0...0> for a batch of B
    bitstrings (array of shape (B, n_qubits)): one network whose projector
    leaves share an extra open label of extent B (a batch label), so the
    result is the vector of the B amplitudes."""
    bits = np.asarray(bitstrings, dtype=np.int64)
    B = bits.shape[0]
    base = circuit_network(circ, open_qubits=range(circ.n_qubits))
    batch = len(base.extents)
    leaves = list(base.leaves)
    labels = list(base.labels)
    for q, wire in enumerate(base.open):
        v = np.zeros((B, 2), dtype=np.complex128)
        v[np.arange(B), bits[:, q]] = 1.0
        leaves.append(v)
        labels.append((batch, wire))
    extents = np.concatenate([base.extents, np.array([B], dtype=np.int64)])
    return Network(leaves, labels, extents, (batch,))
