"""Helpers shared by the GPU tests (device buffers from torch, comparisons)."""
import numpy as np


def rel_fro(got, ref):
    got = np.asarray(got, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def to_dev(torch, x: np.ndarray):
    """complex64 numpy array -> contiguous torch CUDA tensor (same bytes)."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy()
