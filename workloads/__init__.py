"""Seeded synthetic inputs for the tensor-network path executor.

This package only *generates* inputs: networks (leaf tensors, mode labels,
extents, open labels), contraction paths and slicing choices.  It holds none
of the contraction arithmetic.  Both the oracle and the HIP path consume what
it produces, so it must never import either of them.

Contents
  network   -- the Network / Path containers and the .tnz file format
  circuits  -- Haar-random quantum circuits and their tensor networks
  grids     -- closed 2D random tensor networks (many-body-dynamics shaped)
  pairs     -- single large pairwise contractions with permuted stored layouts
  paths     -- greedy min-size path finder, random-greedy paths, greedy slicer
  configs   -- the named benchmark workloads built from the above
"""
from .network import Network, Path, save_tnz, load_tnz  # noqa: F401
