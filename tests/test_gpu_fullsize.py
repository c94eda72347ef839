"""Parity at the benchmark sizes, in the launch configuration bench.py times.

pair30 (A 2^30, B 2^28, C 2^30 complex64): the oracle cannot hold the whole
product, so the result is checked
  * everywhere at once by Freivalds' test with two independent random
    complex vectors r: ||C r - A (B^T r)|| / ||A (B^T r)||.  C r - A (B^T r)
    = E r for the error matrix E, so for random r the ratio estimates the
    relative Frobenius error of C, which float32 accumulation puts near
    sqrt(2k / 6) * 2^-24 ~ 4e-6 for k = 2^14; the bound is 1e-5;
  * exactly on 64 sampled full rows against numpy complex128 products of
    the same operand rows (relative Frobenius error <= 1e-5, and every
    element within the float32 accumulation bound of its row and column,
    8 sqrt(k) 2^-24 ||A_i|| ||B_j||), 8 of them also through the oracle's
    own contraction of the sub-network with those M labels fixed.
pair_batch (64 x 20/18 modes): the whole result against the oracle, in norm
and elementwise (one element among 16.7 M off by a few per cent fails).
circuit40 (65,536 slices): single seeded slices and a batched chunk of 256
slices against the oracle's per-slice contraction.
"""
import numpy as np
import pytest

from tests.gpu_util import U32, assert_close, rel_fro

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import contract as oc  # noqa: E402
from paper_2606_01852_amd import tnc  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.network import Network, Path  # noqa: E402


def make_ctx(gib):
    arena = torch.empty(int(gib * (1 << 30)), dtype=torch.uint8, device="cuda")
    c = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr(),
                    stream=torch.cuda.current_stream().cuda_stream)
    c._arena = arena
    return c


def test_pair30_full_size_freivalds_and_rows():
    print("pair30: generating inputs", flush=True)
    net, path = configs.pair30()
    a, b = net.leaves
    la, lb = net.labels
    M, K, N = list(range(16)), list(range(16, 30)), list(range(30, 44))
    ctx = make_ctx(18.5)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.leaves)
    plan = tnc.Plan(tn, path.pairs)
    out = torch.empty(plan.info.n_result, dtype=torch.complex64, device="cuda")
    print("pair30: contracting", flush=True)
    tnc.tnc_contract_async(plan.handle, 0, 1, out.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    C = out.cpu().numpy().reshape(2 ** 16, 2 ** 14)
    del out
    print("pair30: Freivalds", flush=True)
    Am = np.transpose(a, [la.index(l) for l in M + K]).reshape(2 ** 16, 2 ** 14)
    Bm = np.transpose(b, [lb.index(l) for l in N + K]).reshape(2 ** 14, 2 ** 14)
    rng = np.random.Generator(np.random.PCG64(31))
    for trial in range(2):
        r = (rng.standard_normal(2 ** 14) + 1j * rng.standard_normal(2 ** 14)) / np.sqrt(2)
        Btr = Bm.astype(np.complex128).T @ r                      # sum_j B[j, l] r[j]
        lhs = np.empty(2 ** 16, dtype=np.complex128)
        rhs = np.empty(2 ** 16, dtype=np.complex128)
        for i0 in range(0, 2 ** 16, 4096):
            lhs[i0:i0 + 4096] = C[i0:i0 + 4096].astype(np.complex128) @ r
            rhs[i0:i0 + 4096] = Am[i0:i0 + 4096].astype(np.complex128) @ Btr
        frei = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
        print(f"pair30: Freivalds ratio (trial {trial}) {frei:.2e}", flush=True)
        assert frei <= 1e-5
    # 64 sampled rows against numpy complex128 products of the same operand
    # rows, in norm and elementwise; 8 of them also through the oracle's own
    # contraction of the sub-network (fixed M labels)
    rows = np.sort(rng.choice(2 ** 16, 64, replace=False))
    A64 = Am[rows].astype(np.complex128)
    ref64 = np.empty((64, 2 ** 14), dtype=np.complex128)
    nb = np.empty(2 ** 14)
    for j0 in range(0, 2 ** 14, 2048):
        Bc = Bm[j0:j0 + 2048].astype(np.complex128)
        ref64[:, j0:j0 + 2048] = A64 @ Bc.T
        nb[j0:j0 + 2048] = np.linalg.norm(Bc, axis=1)
    bound = 8 * np.sqrt(2 ** 14) * U32 * np.linalg.norm(A64, axis=1)[:, None] * nb[None, :]
    got64 = C[rows].astype(np.complex128)
    err = rel_fro(got64, ref64)
    ratio = float(np.max(np.abs(got64 - ref64) / bound))
    print(f"pair30: 64 rows: relative Frobenius error {err:.2e}; largest element error / its bound {ratio:.3f}",
          flush=True)
    assert err <= 1e-5 and ratio <= 1.0
    for i in rows[:8]:
        digits = [(int(i) >> (15 - q)) & 1 for q in range(16)]
        fix = dict(zip(M, digits))
        idx = tuple(fix[l] if l in fix else slice(None) for l in la)
        sub = Network([np.ascontiguousarray(a[idx]), b], [tuple(l for l in la if l not in fix), lb],
                      net.extents, tuple(N))
        ref = oc.contract(sub, Path(path.pairs, ())).reshape(-1)
        assert rel_fro(C[i], ref) <= 1e-5, i
    plan.close()
    tn.close()
    ctx.close()


def test_pair_batch_full_size():
    net, path = configs.pair_batch(64)
    ctx = make_ctx(2)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.leaves)
    plan = tnc.Plan(tn, path.pairs)
    out = torch.empty(plan.info.n_result, dtype=torch.complex64, device="cuda")
    tnc.tnc_contract_async(plan.handle, 0, 1, out.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oc.contract(net, path).reshape(-1)
    err = assert_close(got, ref, what="pair_batch")
    print(f"pair_batch: err {err:.2e}", flush=True)


def test_circuit40_sampled_slices():
    """Per-slice amplitudes of a random circuit are Porter-Thomas distributed:
    many slices sit far below the typical magnitude, where float32
    cancellation alone exceeds 1e-5 of |z| (the oracle's own complex64
    evaluation along this path does).  Errors are therefore bounded by 1e-5
    of the root-mean-square amplitude of the sampled ensemble, and the
    relative errors are printed as the measured distribution."""
    net, path = configs.circuit40()
    ctx = make_ctx(16)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, path.sliced)
    assert plan.info.n_slices == 65536
    rng = np.random.Generator(np.random.PCG64(1003))
    sample = [int(x) for x in rng.choice(65536, 24, replace=False)]
    got = np.array([complex(plan.contract(s, 1)[0]) for s in sample])
    ref = np.array([complex(oc.contract(net, path, slices=[s])) for s in sample])
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"circuit40 slices: relative errors median {np.median(rel):.2e} max {rel.max():.2e}; "
          f"max error / rms amplitude {np.max(np.abs(got - ref)) / rms:.2e}", flush=True)
    assert np.max(np.abs(got - ref)) <= 1e-5 * rms
    # a batched chunk of 256 slices, summed in FP64 on the device
    refs = np.array([complex(oc.contract(net, path, slices=[s])) for s in range(256, 512)])
    tot = complex(plan.contract(256, 256)[0])
    scale = np.sqrt(np.sum(np.abs(refs) ** 2))
    err = abs(tot - refs.sum())
    print(f"circuit40 slices [256, 512): |err| / |sum| {err / abs(refs.sum()):.2e}, "
          f"|err| / sqrt(sum |z_s|^2) {err / scale:.2e}", flush=True)
    assert err <= 1e-5 * scale
