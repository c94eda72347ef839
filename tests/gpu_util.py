"""Helpers shared by the GPU tests (device buffers from torch, comparisons).

Every tensor comparison checks two things:
  * the relative Frobenius error (the tolerance norm of the complex64 path);
  * an elementwise bound, so that one wrong element among millions cannot
    hide inside a norm.  For a single GEMM it is the float32 accumulation
    bound of that element, c * sqrt(k) * 2^-24 * ||A_i|| * ||B_j|| (row i of
    A and row j of B, both K-contiguous); for whole paths, where errors pass
    through many steps, every element must lie within elem * tol * max|ref|.
"""
import numpy as np

U32 = 2.0 ** -24     # float32 unit roundoff


def rel_fro(got, ref):
    got = np.asarray(got, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def assert_close(got, ref, tol=1e-5, elem=8.0, what=""):
    """Relative Frobenius error <= tol and max |got - ref| <= elem * tol *
    max |ref| (an error of a few per cent in any one element fails)."""
    got = np.asarray(got, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    err = rel_fro(got, ref)
    assert err <= tol, f"{what}: relative Frobenius error {err:.3e} > {tol:.1e}"
    worst = float(np.max(np.abs(got - ref))) if got.size else 0.0
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    assert worst <= elem * tol * scale, \
        f"{what}: max elementwise error {worst:.3e} > {elem} * {tol:.1e} * max|ref| {scale:.3e}"
    return err


def gemm_elem_bound(A, B, c=8.0):
    """Per-element float32 accumulation bound of C[b,i,j] = sum_l A[b,i,l]
    B[b,j,l]: c * sqrt(k) * 2^-24 * ||A[b,i,:]|| * ||B[b,j,:]||.  The
    rounding of the 2k real products and their running sums grows like
    sqrt(k) times the operand norms for data of random signs; c = 8 leaves
    room for the largest of many millions of elements."""
    k = A.shape[-1]
    na = np.linalg.norm(A.astype(np.complex128), axis=-1)        # [h, m]
    nb = np.linalg.norm(B.astype(np.complex128), axis=-1)        # [h, n]
    return c * np.sqrt(k) * U32 * na[..., :, None] * nb[..., None, :]


def assert_gemm_close(got, ref, A, B, tol=1e-5, c=8.0, what=""):
    """A GEMM result against its complex128 reference: relative Frobenius
    error <= tol, and every element within its own accumulation bound."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    err = rel_fro(got, ref)
    assert err <= tol, f"{what}: relative Frobenius error {err:.3e} > {tol:.1e}"
    bound = gemm_elem_bound(A, B, c).reshape(got.shape) + 1e-30
    ratio = np.abs(got - ref) / bound
    worst = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert ratio[worst] <= 1.0, f"{what}: element {worst} off by {abs(got - ref)[worst]:.3e}, bound {bound[worst]:.3e}"
    return err


def split_elem_bound(A, B):
    """Per-element bound of the split-bf16x3 product against the exact one:
    every real product a b loses at most 3 * 2^-16 |a| |b| (the dropped
    a_lo b_lo and the rounding of the lo parts), and a complex output sums
    four such real products per l: 3 * 2^-16 * sum_l (|ar| + |ai|)(|br| + |bi|)."""
    a = np.abs(A.real) + np.abs(A.imag)
    b = np.abs(B.real) + np.abs(B.imag)
    return 3 * 2.0 ** -16 * np.einsum("...ik,...jk->...ij", a.astype(np.float64), b.astype(np.float64))


def to_dev(torch, x: np.ndarray):
    """complex64 numpy array -> contiguous torch CUDA tensor (same bytes)."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy()
