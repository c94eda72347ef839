"""GPU parity of the two kernels on the hot path, called through the C ABI.

a3 (operand permutation): a bit copy, so the result must be bit-exact with
numpy.transpose; applying the inverse permutation must give back the input.
a4 (batched complex GEMM): compared with a complex128 numpy product; the
tolerance follows from float32 accumulation (unit roundoff 2**-24 times
~sqrt(k) for random data): the 1e-5 relative Frobenius bound of the
complex64 path, and every element within its own accumulation bound
8 sqrt(k) 2^-24 ||A_i|| ||B_j||.  The split-bf16 form is compared with the FP64 emulation of
the same three-product arithmetic (exact products, so only float32
accumulation separates them) and with the exact product (a-priori bound
3 * 2**-16 per real product).
"""
import zlib

import numpy as np
import pytest

from tests.gpu_util import (assert_close, assert_gemm_close, from_dev, gemm_elem_bound, rel_fro,  # noqa: F401
                            split_elem_bound, to_dev)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import split as osp  # noqa: E402
from paper_2606_01852_amd import tnc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    c = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr(),
                    stream=torch.cuda.current_stream().cuda_stream)
    c._arena = arena
    yield c
    c.close()


def cn(rng, shape):
    z = rng.standard_normal(shape + (2,), dtype=np.float32) * np.float32(np.sqrt(0.5))
    return z.view(np.complex64).reshape(shape)


PERM_CASES = [
    ("binary20", (2,) * 20, None),
    ("mixed", (3, 4, 5, 2, 7, 6, 2), None),
    ("tiny", (2, 3, 4), (2, 0, 1)),
    ("common_inner", (2,) * 16 + (8,), "keep_last"),
    ("split_large", (64, 96, 2, 50), (3, 1, 0, 2)),
    ("unit_dims", (1, 2, 1, 2048, 3), (3, 0, 4, 2, 1)),
    ("identity", (4, 4, 4, 4, 4, 4), (0, 1, 2, 3, 4, 5)),
    ("binary24_ragged_tile", (2,) * 12 + (3,) + (2,) * 9, None),
]


@pytest.mark.parametrize("name,ext,perm", PERM_CASES, ids=[c[0] for c in PERM_CASES])
def test_permute_bit_exact(ctx, name, ext, perm):
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(name.encode())))
    r = len(ext)
    if perm is None:
        perm = tuple(int(x) for x in rng.permutation(r))
    elif perm == "keep_last":
        perm = tuple(int(x) for x in rng.permutation(r - 1)) + (r - 1,)
    x = cn(rng, ext)
    print(f"permute {name} ext={ext} perm={perm}", flush=True)
    xd = to_dev(torch, x)
    yd = torch.empty(x.size, dtype=torch.complex64, device="cuda")
    tnc.tnc_permute(ctx.handle, xd.data_ptr(), yd.data_ptr(), ext, perm)
    torch.cuda.synchronize()
    ref = np.ascontiguousarray(np.transpose(x, perm))
    got = from_dev(yd).reshape(ref.shape)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    # the inverse permutation restores the input exactly
    inv = tuple(int(i) for i in np.argsort(perm))
    zd = torch.empty_like(yd)
    tnc.tnc_permute(ctx.handle, yd.data_ptr(), zd.data_ptr(), ref.shape, inv)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(zd).reshape(x.shape).view(np.uint64), x.view(np.uint64))


GEMM_SHAPES = [
    (512, 128, 64, 16),    # exactly one MFMA tile per batch entry
    (24, 200, 100, 50),    # ragged m, n, k on MFMA tiles
    (20, 300, 70, 33),     # odd k: 8-byte loads
    (3, 1000, 500, 600),   # many tiles, batch
    (1, 4096, 1024, 256),
    (5, 10, 3, 4),         # small-shape kernel
    (160, 64, 32, 16),     # smallest MFMA shape
    (1, 128, 64, 16),      # the same shapes with under 2^22 MACs and short K:
    (1, 200, 100, 50),     #   one thread per output
    (2, 300, 70, 33),
    (7, 64, 32, 16),
    (1, 1, 1, 1),
    (3, 1, 1, 5000),       # long-K dot kernel
    (2, 4, 8, 1024),       # long-K dot kernel, several outputs
    (8, 16, 200, 512),     # skinny: MFMA on padded tiles (m < 64)
    (4, 40, 9, 2048),      # skinny in both m and n
]


def ref_gemm(A, B):
    return np.einsum("bik,bjk->bij", A.astype(np.complex128), B.astype(np.complex128))


@pytest.mark.parametrize("form", [tnc.GEMM_4M, tnc.GEMM_3M], ids=["4M", "3M"])
@pytest.mark.parametrize("shape", GEMM_SHAPES, ids=[str(s) for s in GEMM_SHAPES])
def test_cgemm_matches_numpy(ctx, shape, form):
    h, m, n, k = shape
    rng = np.random.Generator(np.random.PCG64(h * 1000003 + m * 1009 + n * 17 + k))
    A, B = cn(rng, (h, m, k)), cn(rng, (h, n, k))
    print(f"cgemm form={form} shape={shape}", flush=True)
    Ad, Bd = to_dev(torch, A), to_dev(torch, B)
    Cd = torch.empty((h, m, n), dtype=torch.complex64, device="cuda")
    torch.view_as_real(Cd).fill_(float("nan"))
    tnc.tnc_batched_cgemm(ctx.handle, h, m, n, k, Ad.data_ptr(), m * k, Bd.data_ptr(), n * k, Cd.data_ptr(),
                          tnc.PREC_C64, form)
    torch.cuda.synchronize()
    got = from_dev(Cd)
    assert np.all(np.isfinite(got.view(np.float32)))
    assert_gemm_close(got, ref_gemm(A, B), A, B, what=f"cgemm {shape}")


def test_cgemm_broadcast_operand(ctx):
    h, m, n, k = 4, 256, 96, 40
    rng = np.random.Generator(np.random.PCG64(77))
    A, B = cn(rng, (h, m, k)), cn(rng, (1, n, k))
    Ad, Bd = to_dev(torch, A), to_dev(torch, B)
    Cd = torch.empty((h, m, n), dtype=torch.complex64, device="cuda")
    tnc.tnc_batched_cgemm(ctx.handle, h, m, n, k, Ad.data_ptr(), m * k, Bd.data_ptr(), 0, Cd.data_ptr())
    torch.cuda.synchronize()
    Bb = np.broadcast_to(B, (h, n, k))
    assert_gemm_close(from_dev(Cd), ref_gemm(A, Bb), A, Bb, what="broadcast B")


def split_emulated_gemm(A, B):
    def prod3(x, y):
        xh, xl = osp.split(x)
        yh, yl = osp.split(y)
        e = lambda p, q: np.einsum("bik,bjk->bij", p, q)
        return e(xh, yh) + e(xh, yl) + e(xl, yh)
    ar, ai = A.real, A.imag
    br, bi = B.real, B.imag
    return (prod3(ar, br) - prod3(ai, bi)) + 1j * (prod3(ar, bi) + prod3(ai, br))


@pytest.mark.parametrize("shape", [(4, 256, 128, 64), (16, 130, 70, 33), (3, 20, 5, 7), (2, 2, 3, 700),
                                   (8, 16, 200, 512), (1, 256, 128, 64)],
                         ids=["tiles", "ragged", "small", "dot", "skinny", "short_k_small"])
def test_cgemm_bf16x3_matches_split_emulation(ctx, shape):
    h, m, n, k = shape
    rng = np.random.Generator(np.random.PCG64(m + n + k))
    A, B = cn(rng, (h, m, k)), cn(rng, (h, n, k))
    print(f"cgemm bf16x3 shape={shape}", flush=True)
    Ad, Bd = to_dev(torch, A), to_dev(torch, B)
    Cd = torch.empty((h, m, n), dtype=torch.complex64, device="cuda")
    tnc.tnc_batched_cgemm(ctx.handle, h, m, n, k, Ad.data_ptr(), m * k, Bd.data_ptr(), n * k, Cd.data_ptr(),
                          tnc.PREC_BF16X3, tnc.GEMM_4M)
    torch.cuda.synchronize()
    got = from_dev(Cd)
    emu = split_emulated_gemm(A, B)
    exact = ref_gemm(A, B)
    # the emulation's products are exact: only float32 accumulation (of three
    # times as many terms) separates them
    assert_gemm_close(got, emu, A, B, what=f"bf16x3 {shape} vs emulation")
    # against the exact product: a-priori bound of the split (3 * 2**-16 per
    # real product), per element and in norm, far looser than the emulation
    bound = split_elem_bound(A, B) + 2 * gemm_elem_bound(A, B)
    assert np.all(np.abs(got - exact) <= bound)
    assert rel_fro(got, exact) <= 3 * 2.0 ** -16 * 4


def split_3m_emulated_gemm(A, B):
    """The oracle's 3M split step over batch label 0 (A[b, i, l] B[b, j, l])."""
    z, lz = osp.split_step_3m(A.astype(np.complex128), [0, 1, 3], B.astype(np.complex128), [0, 2, 3], {0, 1, 2})
    assert lz == [0, 1, 2]
    return z


@pytest.mark.parametrize("shape", [(4, 256, 128, 64), (16, 130, 70, 33), (8, 16, 200, 512), (1, 512, 256, 1000),
                                   (16, 200, 100, 17)],
                         ids=["tiles", "ragged_odd_k", "skinny", "long_k", "short_odd_k"])
def test_cgemm_bf16x3_3m_matches_split_emulation(ctx, shape):
    """Split precision in the 3M form (three split real products, nine bf16
    products per complex product) on MFMA steps: within float32 accumulation
    of the oracle's 3M split emulation, per element, and within twice the
    split's a-priori bound of the exact product (T3's operands are sums of
    two parts)."""
    h, m, n, k = shape
    rng = np.random.Generator(np.random.PCG64(3 * m + n + k))
    A, B = cn(rng, (h, m, k)), cn(rng, (h, n, k))
    print(f"cgemm bf16x3 3M shape={shape}", flush=True)
    Ad, Bd = to_dev(torch, A), to_dev(torch, B)
    Cd = torch.empty((h, m, n), dtype=torch.complex64, device="cuda")
    torch.view_as_real(Cd).fill_(float("nan"))
    tnc.tnc_batched_cgemm(ctx.handle, h, m, n, k, Ad.data_ptr(), m * k, Bd.data_ptr(), n * k, Cd.data_ptr(),
                          tnc.PREC_BF16X3, tnc.GEMM_3M)
    torch.cuda.synchronize()
    got = from_dev(Cd)
    emu = split_3m_emulated_gemm(A, B)
    assert_gemm_close(got, emu, A, B, what=f"bf16x3 3M {shape} vs emulation")
    exact = ref_gemm(A, B)
    bound = 2 * split_elem_bound(A, B) + 2 * gemm_elem_bound(A, B)
    assert np.all(np.abs(got - exact) <= bound)
    assert rel_fro(got, exact) <= 3 * 2.0 ** -16 * 8
    # a different sequence of roundings than the 4M split form
    assert not np.array_equal(got, split_emulated_gemm(A, B).astype(np.complex64))


@pytest.mark.parametrize("variant", range(7))
@pytest.mark.parametrize("kind", ["4M", "3M", "bf16x3", "bf16x3_3M"])
def test_every_tile_variant(ctx, variant, kind):
    """Each MFMA workgroup shape on an interior-tile shape and a ragged one
    (the 3M split form runs a forced variant 3 on its (4,2) tile)."""
    prec = tnc.PREC_BF16X3 if kind.startswith("bf16x3") else tnc.PREC_C64
    form = tnc.GEMM_3M if kind.endswith("3M") else tnc.GEMM_4M
    tnc.tnc_ctx_set_gemm_variant(ctx.handle, variant)
    try:
        for (h, m, n, k) in ((2, 512, 256, 64), (3, 333, 111, 70)):
            rng = np.random.Generator(np.random.PCG64(variant * 100 + m))
            A, B = cn(rng, (h, m, k)), cn(rng, (h, n, k))
            print(f"variant {variant} {kind} shape {(h, m, n, k)}", flush=True)
            Ad, Bd = to_dev(torch, A), to_dev(torch, B)
            Cd = torch.empty((h, m, n), dtype=torch.complex64, device="cuda")
            torch.view_as_real(Cd).fill_(float("nan"))
            tnc.tnc_batched_cgemm(ctx.handle, h, m, n, k, Ad.data_ptr(), m * k, Bd.data_ptr(), n * k,
                                  Cd.data_ptr(), prec, form)
            torch.cuda.synchronize()
            got = from_dev(Cd)
            ref = {"bf16x3": split_emulated_gemm, "bf16x3_3M": split_3m_emulated_gemm}.get(kind, ref_gemm)(A, B)
            assert_gemm_close(got, ref, A, B, what=f"variant {variant} {kind} {(h, m, n, k)}")
    finally:
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)


def test_autotune_keeps_results_and_persists(ctx, tmp_path, monkeypatch):
    from workloads.pairs import pair_network
    from oracle import contract as oc
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TNC_AUTOTUNE_CACHE", str(cache))
    c2 = tnc.Context(0, arena_bytes=512 << 20)
    net, path = pair_network(11, 9, 9, seed=12)
    tn = tnc.Network(c2, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    before = plan.contract()
    tnc.tnc_plan_autotune(plan.handle)
    v = tnc.tnc_plan_get_step(plan.handle, 0).variant
    assert 0 <= v < tnc.tnc_gemm_variant_count()
    after = plan.contract()
    ref = oc.contract(net, path).reshape(-1)
    assert_close(after, ref, what="autotuned")
    assert_close(before, ref, what="default tiles")
    lines = cache.read_text().split()
    assert len(lines) == 8 and int(lines[-1]) == v
    # a new context reads the cache back and assigns the same variant untimed
    c3 = tnc.Context(0, arena_bytes=512 << 20)
    tn3 = tnc.Network(c3, net.labels, net.extents, net.open, net.c64().leaves)
    plan3 = tnc.Plan(tn3, path.pairs)
    assert tnc.tnc_plan_get_step(plan3.handle, 0).variant == v


def test_device_calibration(ctx):
    """The measured FP32 MFMA rate and copy bandwidth are plausible for the
    device (they feed the distribution cost model and the bench's measured
    ceilings)."""
    hw = tnc.tnc_device_calibrate(ctx.handle)
    print(f"calibration: FP32 MFMA {hw.flops_per_s / 1e12:.1f} TFLOP/s, copy {hw.hbm_bytes_per_s / 1e9:.0f} GB/s",
          flush=True)
    assert 20e12 < hw.flops_per_s < 400e12
    assert 0.5e12 < hw.hbm_bytes_per_s < 20e12
    host = tnc.Context(-1)     # keep the handle alive across the call
    with pytest.raises(tnc.TncError):
        tnc.tnc_device_calibrate(host.handle)


def test_bad_choices_are_refused_before_any_launch(ctx):
    """On a device context, unknown precisions, GEMM forms and output types
    and malformed permutes come back as TNC_E_ARG and leave the output
    untouched (nothing was launched)."""
    import ctypes as C
    L = tnc.lib()
    a = to_dev(torch, np.ones((4, 8), dtype=np.complex64))
    c = torch.full((4, 4), 7.0 + 0j, dtype=torch.complex64, device="cuda")
    for prec, form in ((7, tnc.GEMM_4M), (tnc.PREC_C64, -3)):
        st = L.tnc_batched_cgemm(ctx.handle, 1, 4, 4, 8, a.data_ptr(), 0, a.data_ptr(), 0, c.data_ptr(), prec, form)
        assert st == tnc.E_ARG
    ext = np.array([4, 8], dtype=np.int64)
    for perm, e in (([1, 1], ext), ([1, 0], np.array([1 << 31, 1 << 31], dtype=np.int64))):
        p = np.array(perm, dtype=np.int32)
        st = L.tnc_permute(ctx.handle, a.data_ptr(), c.data_ptr(), 2, e.ctypes.data_as(C.POINTER(C.c_int64)),
                           p.ctypes.data_as(C.POINTER(C.c_int32)))
        assert st == tnc.E_ARG
    tn = tnc.Network(ctx, [(0, 1), (1, 2)], np.array([4, 8, 4], dtype=np.int64), (0, 2),
                     [np.ones((4, 8), np.complex64), np.ones((8, 4), np.complex64)])
    plan = tnc.Plan(tn, [(0, 1)])
    assert L.tnc_contract_async(plan.handle, 0, 1, c.data_ptr(), 5) == tnc.E_ARG
    torch.cuda.synchronize()
    assert bool((c == (7.0 + 0j)).all())
    plan.close()
    tn.close()
