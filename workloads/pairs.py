"""Single large pairwise contractions with permuted stored layouts.

A has modes M u K, B has modes N u K (all extents 2 unless given); the
result order is [M ascending || N ascending].  Labels: M = 0..nm-1,
K = nm..nm+nk-1, N = nm+nk..nm+nk+nn-1.  The stored mode order of A is a
seeded random permutation of M u K and that of B a seeded random
permutation of N u K, so that an operand permutation precedes the GEMM.
Entries are i.i.d. complex Gaussian with E|z|^2 = 1, generated directly in
complex64.  With ``batch`` > 1 a batch label (extent ``batch``) leads both
operands and the result: ``batch`` independent contractions that share one
label structure and one permutation but have independent entries.
"""
from __future__ import annotations

import numpy as np

from .network import Network, Path


def _cn64(rng: np.random.Generator, n: int) -> np.ndarray:
    re_im = rng.standard_normal(2 * n, dtype=np.float32)
    re_im *= np.float32(np.sqrt(0.5))
    return re_im.view(np.complex64)


def pair_network(nm: int, nk: int, nn: int, seed: int, batch: int = 1, ext: int = 2):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = list(range(nm))
    K = list(range(nm, nm + nk))
    N = list(range(nm + nk, nm + nk + nn))
    n_lab = nm + nk + nn
    a_order = [int(x) for x in rng.permutation(M + K)]
    b_order = [int(x) for x in rng.permutation(N + K)]
    extents = np.full(n_lab + (1 if batch > 1 else 0), ext, dtype=np.int64)
    a_lab, b_lab, out = tuple(a_order), tuple(b_order), tuple(M + N)
    if batch > 1:
        z = n_lab
        extents[z] = batch
        a_lab, b_lab, out = (z,) + a_lab, (z,) + b_lab, (z,) + out
    a_shape = tuple(int(extents[l]) for l in a_lab)
    b_shape = tuple(int(extents[l]) for l in b_lab)
    a = _cn64(rng, int(np.prod(a_shape))).reshape(a_shape)
    b = _cn64(rng, int(np.prod(b_shape))).reshape(b_shape)
    net = Network([a, b], [a_lab, b_lab], extents, out)
    return net, Path(np.array([[0, 1]], dtype=np.int32), ())
