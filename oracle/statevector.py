"""Brute-force state-vector simulation of a gate circuit.

ORACLE -- test infrastructure only (see the package header).

An independent route to circuit amplitudes: start from |0...0>, apply every
gate in circuit order to the full 2**n complex128 state, read the amplitude
<x|psi>.  Qubit 0 is the most significant bit of the state index.  A 1q gate
is U[out, in]; a 2q gate on (q1, q2) is the 4x4 matrix with row index
2*o1 + o2.  Practical up to ~26 qubits.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def run(n_qubits: int, gates) -> np.ndarray:
    psi = np.zeros((2,) * n_qubits, dtype=np.complex128)
    psi[(0,) * n_qubits] = 1.0
    for qs, u in gates:
        u = np.asarray(u, dtype=np.complex128)
        if len(qs) == 1:
            (q,) = qs
            psi = np.moveaxis(np.tensordot(u, psi, axes=([1], [q])), 0, q)
        else:
            q1, q2 = qs
            g = u.reshape(2, 2, 2, 2)
            psi = np.moveaxis(np.tensordot(g, psi, axes=([2, 3], [q1, q2])), [0, 1], [q1, q2])
    return psi


def amplitude(n_qubits: int, gates, bits: Sequence[int]) -> complex:
    return complex(run(n_qubits, gates)[tuple(int(b) for b in bits)])
