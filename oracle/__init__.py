"""Oracle: a plain, slow, obviously correct CPU reference (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  The product path never calls it, and it
never imports the product path: the two share no code, only the seeded input
generators in ``workloads``.

Everything here computes in float64 / complex128 from the definitions in the
paper (arXiv 2606.01852, "Parallelizing Large-Scale Tensor Network
Contraction on Multiple GPUs"):

  contract     exact contraction of a network along a pairwise path, summing
               over sliced labels (Sec. II-A, II-B, II-C)
  statevector  brute-force state-vector simulation of a gate circuit: an
               independent check of circuit amplitudes
  reorder      the GEMM-oriented mode-reordering backward pass (Sec. IV-A)
  costs        per-step m, n, k and the path costs C_t, C_s, C_m
               (Sec. II-B, Eq. (1)-(3)); 8 real FLOPs per complex MAC
  split        bf16 hi/lo split by round-to-nearest-even bit manipulation and
               the three-product emulation of a split-precision product, in
               the 4M and the 3M complex form
  distplan     keep-or-redistribute choices along a use-chain by exhaustive
               enumeration under the cost model (Sec. IV-B, Eq. (4)-(7))
"""
