"""The benchmark workloads as seeded synthetic inputs.

They stand in for the paper's instances (random quantum circuits and
many-body lattices, Sec. V), which are not used.

Seeds follow ``PCG64(1000 + workload id)``; serving request ``i`` uses
``PCG64(5000 + i)``.

  circuit12   12-qubit 3x4 grid circuit, depth 8, closed amplitude network
  pair30      A 30 modes x B 28 modes, 14 shared, output 2^30 entries
  pair_batch  64 independent 20-mode x 18-mode contractions, 10 shared
  grid8       closed 8x8 grid network, bond 4, contracted to a scalar
  circuit40   40-qubit 5x8 grid circuit, depth 12, 16 sliced labels
  serve_pool  random grid circuits of 20..48 qubits, depth 8..14
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .circuits import circuit_network, random_circuit
from .grids import random_grid_network
from .network import Network, Path
from .pairs import pair_network
from .paths import greedy_path, greedy_slice, path_cost


def circuit12(open_qubits=()) -> Tuple[Network, Path]:
    circ = random_circuit(3, 4, 8, seed=1000)
    net = circuit_network(circ, open_qubits=open_qubits)
    return net, greedy_path(net)


def circuit12_circuit():
    return random_circuit(3, 4, 8, seed=1000)


def pair30(scale: int = 0) -> Tuple[Network, Path]:
    """``scale`` > 0 removes that many modes from each of M, K and N (a
    smaller instance with the same structure, for tests)."""
    return pair_network(16 - scale, 14 - scale, 14 - scale, seed=1001)


def pair_batch(batch: int = 64, scale: int = 0) -> Tuple[Network, Path]:
    return pair_network(10 - scale, 10 - scale, 8 - scale, seed=1101, batch=batch)


def grid8(rows: int = 8, cols: int = 8, bond: int = 4) -> Tuple[Network, Path]:
    net = random_grid_network(rows, cols, bond, seed=1002)
    p = greedy_path(net)
    big, _ = path_cost(net, p.pairs)
    if big > 2 ** 32:
        raise RuntimeError(f"greedy path's largest intermediate {big} exceeds 2^32")
    return net, p


def circuit40(n_sliced: int = 16, rows: int = 5, cols: int = 8, depth: int = 12,
              seed: int = 1003) -> Tuple[Network, Path]:
    circ = random_circuit(rows, cols, depth, seed=seed)
    net = circuit_network(circ)
    p = greedy_path(net)
    sl = greedy_slice(net, p.pairs, n_sliced=n_sliced)
    return net, Path(p.pairs, sl)


def serve_request_spec(i: int):
    """(rows, cols, depth, log4 slices, precision) of serving pool entry i."""
    rng = np.random.Generator(np.random.PCG64(5000 + i))
    while True:
        rows = int(rng.choice([4, 5, 6]))
        cols = int(rng.integers(4, 9))
        if 20 <= rows * cols <= 48:
            break
    depth = int(rng.integers(8, 15))
    j = int(rng.integers(0, 7))
    prec = int(rng.integers(0, 2))
    return rows, cols, depth, j, prec


def serve_request_circuit(i: int, max_log2_ops: float = 43.0):
    """(circuit, network, path with 4**j slices, precision flag) of pool
    entry i.  Slices are chosen greedily; the request's planned operation
    count is capped at 2**max_log2_ops by lowering the depth."""
    rows, cols, depth, j, prec = serve_request_spec(i)
    while True:
        circ = random_circuit(rows, cols, depth, seed=5000 + i)
        net = circuit_network(circ)
        p = greedy_path(net)
        sl = greedy_slice(net, p.pairs, n_sliced=2 * j) if j else ()
        big, ops = path_cost(net, p.pairs, sl)
        n_sl = 4 ** j
        if math.log2(max(ops, 1) * n_sl * 8) <= max_log2_ops or depth <= 4:   # exact for ints past 2^63
            return circ, net, Path(p.pairs, sl), prec
        depth -= 1


def serve_request(i: int, max_log2_ops: float = 43.0) -> Tuple[Network, Path, int]:
    """Network, path (with 4**j slices) and precision flag of pool entry i."""
    _, net, path, prec = serve_request_circuit(i, max_log2_ops)
    return net, path, prec
