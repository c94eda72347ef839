"""GPU parity of whole path executions (C ABI) against the FP64 oracle.

Each case runs the plan on the GPU and compares with the oracle on the same
seeded inputs (complex64 leaves upcast to complex128):
  * scalars: |z - z_ref| / |z_ref| <= 1e-5; tensors: relative Frobenius
    error <= 1e-5 (complex64 path) and every element within 8e-5 of the
    largest reference element (so one wrong element cannot hide in the norm);
  * split-bf16 paths: against the oracle's split emulation (same products,
    FP64 sums, complex64 storage per step) within 1e-5: only float32
    accumulation separates them, the same error class as the complex64 path;
    against the exact value within max(1e-5, 4 * 2**-16 * D), the a-priori
    split bound (3 * 2**-16 per real product) compounded once per level of
    the contraction tree (depth D of the root);
  * circuit amplitudes also against the brute-force state vector.
"""
import numpy as np
import pytest

from tests.gpu_util import assert_close, rel_fro

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import contract as oc  # noqa: E402
from oracle import split as osp  # noqa: E402
from oracle import statevector as osv  # noqa: E402
from paper_2606_01852_amd import tnc  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.circuits import circuit_network, random_circuit  # noqa: E402
from workloads.grids import prescale_log2, random_grid_network  # noqa: E402
from workloads.network import Network, Path  # noqa: E402
from workloads.pairs import pair_network  # noqa: E402
from workloads.paths import greedy_path, greedy_slice  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    arena = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    c = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr(),
                    stream=torch.cuda.current_stream().cuda_stream)
    c._arena = arena
    yield c
    c.close()


def tree_depth(n_leaves, pairs):
    depth = [0] * n_leaves
    for a, b in pairs:
        depth.append(1 + max(depth[int(a)], depth[int(b)]))
    return depth[-1]


def split_tols(net, path):
    D = tree_depth(net.n_leaves, path.pairs)
    return 1e-5, max(1e-5, 4 * 2.0 ** -16 * D)


def run(ctx, net, path, prec=tnc.PREC_C64, form=tnc.GEMM_4M, first=0, count=None, max_chunk=None):
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
    if max_chunk is not None:
        tnc.tnc_plan_set_max_chunk(plan.handle, max_chunk)
        plan.info = tnc.tnc_plan_get_info(plan.handle)
    out = plan.contract(first, count)
    shape = tuple(int(net.extents[l]) for l in net.open)
    return out.reshape(shape) if shape else complex(out[0]), plan, tn


@pytest.mark.parametrize("form", [tnc.GEMM_4M, tnc.GEMM_3M], ids=["4M", "3M"])
def test_circuit12_amplitude(ctx, form):
    circ = configs.circuit12_circuit()
    net, path = configs.circuit12()
    print("circuit12 amplitude", form, flush=True)
    z, _, _ = run(ctx, net, path, form=form)
    ref = complex(oc.contract(net, path))
    sv = osv.amplitude(circ.n_qubits, circ.gates, circ.bitstring)
    print(f"circuit12 {form}: err vs oracle {abs(z - ref) / abs(ref):.2e}")
    assert abs(z - ref) <= 1e-5 * abs(ref)
    assert abs(z - sv) <= 1e-5 * abs(sv)


def test_circuit12_all_amplitudes_unitarity(ctx):
    circ = configs.circuit12_circuit()
    net = circuit_network(circ, open_qubits=range(12))
    path = greedy_path(net)
    print("circuit12 all amplitudes", flush=True)
    amps, plan, _ = run(ctx, net, path)
    ref = osv.run(12, circ.gates)
    assert_close(amps, ref)
    norm2 = tnc.tnc_plan_result_norm2(plan.handle)
    assert abs(norm2 - 1.0) <= 1e-5
    assert abs(norm2 - float(np.sum(np.abs(amps) ** 2))) <= 1e-12


def test_circuit12_sliced_and_chunking_invariance(ctx):
    net, path = configs.circuit12()
    sl = greedy_slice(net, path.pairs, n_sliced=4)
    p = Path(path.pairs, sl)
    ref = complex(oc.contract(net, p))
    vals = []
    for mc in (1, 2, 16):
        print("circuit12 sliced, max_chunk", mc, flush=True)
        z, plan, _ = run(ctx, net, p, max_chunk=mc)
        assert plan.info.max_chunk == mc
        vals.append(z)
        assert abs(z - ref) <= 1e-5 * abs(ref)
    assert max(abs(v - vals[0]) for v in vals) <= 1e-13 * abs(vals[0])
    # partial ranges and single slices
    z3, _, _ = run(ctx, net, p, first=3, count=9)
    ref3 = complex(oc.contract(net, p, slices=range(3, 12)))
    assert abs(z3 - ref3) <= 1e-5 * abs(ref3)
    z7, _, _ = run(ctx, net, p, first=7, count=1)
    ref7 = complex(oc.contract(net, p, slices=[7]))
    assert abs(z7 - ref7) <= 1e-5 * abs(ref7)


def test_circuit12_split_precision(ctx):
    net, path = configs.circuit12()
    print("circuit12 bf16x3", flush=True)
    z, _, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3)
    emu = complex(oc.contract(net, path, step=osp.split_step))
    exact = complex(oc.contract(net, path))
    t_emu, t_exact = split_tols(net, path)
    print(f"depth {tree_depth(net.n_leaves, path.pairs)}: err vs emulation {abs(z - emu) / abs(emu):.2e} "
          f"(tol {t_emu:.1e}), vs exact {abs(z - exact) / abs(exact):.2e} (tol {t_exact:.1e})")
    assert abs(z - emu) <= t_emu * abs(emu)
    assert abs(z - exact) <= t_exact * abs(exact)


def test_circuit20_sliced_sum_matches_statevector(ctx):
    circ = random_circuit(4, 5, 10, seed=77)
    net = circuit_network(circ)
    path = greedy_path(net)
    sl = greedy_slice(net, path.pairs, n_sliced=6)
    p = Path(path.pairs, sl)
    print("circuit20 sliced", sl, flush=True)
    z, plan, _ = run(ctx, net, p)
    # the state vector with the same complex64-rounded gates the GPU uses,
    # so that only the arithmetic differs
    gates64 = [(q, u.astype(np.complex64).astype(np.complex128)) for q, u in circ.gates]
    sv = osv.amplitude(20, gates64, circ.bitstring)
    ref = complex(oc.contract(net, p))
    assert plan.info.n_slices == 64
    print(f"circuit20 sliced: err vs state vector {abs(z - sv) / abs(sv):.2e}, vs oracle {abs(z - ref) / abs(ref):.2e}")
    assert abs(ref - sv) <= 1e-12 * abs(sv)
    assert abs(z - sv) <= 1e-5 * abs(sv)
    for s in (0, 17, 63):
        zs, _, _ = run(ctx, net, p, first=s, count=1)
        rs = complex(oc.contract(net, p, slices=[s]))
        assert abs(zs - rs) <= 1e-5 * abs(rs)


def prescaled_grid(rows, cols, bond, seed):
    g = random_grid_network(rows, cols, bond, seed=seed)
    e = prescale_log2(g.labels)
    leaves = [x * 2.0 ** int(k) for x, k in zip(g.leaves, e)]
    return Network(leaves, g.labels, g.extents, ()), int(e.sum())


@pytest.mark.parametrize("prec, form", [(tnc.PREC_C64, tnc.GEMM_4M), (tnc.PREC_BF16X3, tnc.GEMM_4M),
                                        (tnc.PREC_BF16X3, tnc.GEMM_3M)], ids=["c64", "bf16x3", "bf16x3_3M"])
def test_grid8_bond4(ctx, prec, form):
    """grid8 (prescaled, 63 steps).  Split precision in the 3M form runs
    its MFMA steps as three split real products and its small (VALU) steps
    in the 4M form: the emulation takes each step's form from the plan.
    Its tolerance against the emulation is three times the 4M form's: the
    imaginary part comes from three float32 accumulators (T3's over sums of
    two parts, up to twice the operand norms) instead of one over 2k terms,
    about 4 / sqrt(2) times the accumulation error (single GEMMs: 1-5e-7 of
    the emulation in either form)."""
    net, shift = prescaled_grid(8, 8, 4, seed=1002)
    path = greedy_path(net)
    print("grid8 prec", prec, "form", form, flush=True)
    z, plan, _ = run(ctx, net, path, prec=prec, form=form)
    exact = complex(oc.contract(net, path))
    if prec == tnc.PREC_C64:
        print(f"grid8 c64: err vs oracle {abs(z - exact) / abs(exact):.2e}")
        assert abs(z - exact) <= 1e-5 * abs(exact)
    else:
        kinds = iter([plan.step(s).kernel for s in range(len(path.pairs))])
        if form == tnc.GEMM_3M:
            def step(x, la, y, lb, keep):   # steps come in path order
                return (osp.split_step_3m if next(kinds) == 0 else osp.split_step)(x, la, y, lb, keep)
        else:
            step = osp.split_step
        emu = complex(oc.contract(net, path, step=step))
        t_emu, t_exact = split_tols(net, path)
        if form == tnc.GEMM_3M:
            t_emu *= 3
            t_exact *= 2   # T3's operands are sums of two parts
        print(f"grid8 bf16x3: err vs emulation {abs(z - emu) / abs(emu):.2e} (tol {t_emu:.1e}), "
              f"vs exact {abs(z - exact) / abs(exact):.2e} (tol {t_exact:.1e})")
        assert abs(z - emu) <= t_emu * abs(emu)
        assert abs(z - exact) <= t_exact * abs(exact)
    # the unscaled value is tiny but representable in FP64
    assert 0 < abs(z) * 2.0 ** -shift < 1e-20


def test_grid8_bf16x3_wide_tile_permuted_stores(ctx):
    """Split-bf16x3's 256 x 128 tile (wide waves, one accumulator set) forced
    on every MFMA step of grid8, most of them stored in consumer order:
    within the split bounds of the emulation and of the exact value."""
    net, shift = prescaled_grid(8, 8, 4, seed=1002)
    path = greedy_path(net)
    tnc.tnc_ctx_set_gemm_variant(ctx.handle, 3)
    try:
        z, plan, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3)
    finally:
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)
    steps = [tnc.tnc_plan_get_step(plan.handle, s) for s in range(len(path.pairs))]
    assert any(st.kernel == 0 and st.natural == 0 for st in steps)   # MFMA with permuted store
    exact = complex(oc.contract(net, path))
    emu = complex(oc.contract(net, path, step=osp.split_step))
    t_emu, t_exact = split_tols(net, path)
    print(f"grid8 bf16x3 wide tile: err vs emulation {abs(z - emu) / abs(emu):.2e} (tol {t_emu:.1e})", flush=True)
    assert abs(z - emu) <= t_emu * abs(emu)
    assert abs(z - exact) <= t_exact * abs(exact)


PRESPLIT_LEAVES = {
    # extents, stored labels of A and of B
    "canonical": ([64, 65, 66, 64, 200], (0, 1, 4), (2, 3, 4)),
    "permuted": ([64, 65, 64, 66, 1024], (4, 1, 0), (4, 3, 2)),
    "permuted_odd": ([66, 63, 63, 66, 1024], (4, 0, 1), (4, 3, 2)),
    "odd_mn": ([64, 65, 65, 65, 256], (0, 1, 4), (2, 3, 4)),   # n = 4225
}


@pytest.mark.parametrize("leaves", list(PRESPLIT_LEAVES))
@pytest.mark.parametrize("order", ["natural", "interleaved"])
def test_presplit_bf16x3_is_bitwise_the_wide_tile(ctx, order, leaves):
    """Large split-bf16x3 steps split their operands once into bf16 planes
    and stage them global -> LDS directly: one GEMM of 4160 x 4224 x 200
    (ragged against the 256 x 128 tile, k padded to 208), stored row-major
    or in an interleaved consumer order.  With permuted leaves (stored K
    first, M or N labels reversed; 4160 x 4224 x 1024, so that they exceed
    the 2^22-element leaf cache) the leaf permutes write the planes
    themselves (one pass), while the forced wide-wave run permutes them to
    complex64 as usual: "permuted" has even input runs (the 16-byte pair
    kernel), "permuted_odd" input runs of 63 elements (the element-wise
    tiled kernel, 4158 x 4158 x 1024); "odd_mn" an odd n (4160 x 4225 x
    256).  The result is bitwise that of the
    wide-wave kernel (variant 3, forced) and of its hipGraph replays,
    within 1e-5 of the oracle's split emulation, and every element within
    the split bound of the exact product."""
    rng = np.random.Generator(np.random.PCG64(4160))
    ext, la, lb = PRESPLIT_LEAVES[leaves]
    ext = np.array(ext, dtype=np.int64)

    def cn(lab):
        shape = tuple(int(ext[l]) for l in lab)
        x = rng.standard_normal(shape + (2,), dtype=np.float32) * np.float32(np.sqrt(0.5))
        return x.view(np.complex64).reshape(shape)
    out = (0, 1, 2, 3) if order == "natural" else (0, 2, 1, 3)
    net = Network([cn(la), cn(lb)], [la, lb], ext, out)
    path = Path(np.array([[0, 1]], dtype=np.int32), ())
    print(f"presplit bf16x3 {order} {leaves}", flush=True)
    z, plan, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3)
    st = tnc.tnc_plan_get_step(plan.handle, 0)
    assert st.kernel == 0 and st.presplit == 1 and st.split == 1
    assert st.natural == (1 if order == "natural" else 0)
    permuted = leaves.startswith("permuted")
    assert plan.info.n_permutes == (2 if permuted else 0)
    assert st.presplit_fused == (3 if permuted else 0)    # both permutes write planes
    tnc.tnc_ctx_set_gemm_variant(ctx.handle, 3)
    try:
        w, _, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3)
    finally:
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)
    assert np.array_equal(np.asarray(z).view(np.uint64), np.asarray(w).view(np.uint64))
    # captured as a hipGraph (splits and GEMM in the graph), replayed twice
    tnc.tnc_plan_set_graph(plan.handle, True)
    for _ in range(2):
        g = plan.contract().reshape(np.asarray(z).shape)
        assert np.array_equal(g.view(np.uint64), np.asarray(z).view(np.uint64))
    emu = oc.contract(net, path, step=osp.split_step)
    err = assert_close(z, emu, tol=1e-5, what="presplit vs emulation")
    # exact product and the split bound 3 * 2^-16 * sum_l (|ar|+|ai|)(|br|+|bi|) per element
    e0, e1, e2, e3, kk = (int(x) for x in ext)
    A = np.transpose(net.leaves[0], [la.index(x) for x in (0, 1, 4)]).reshape(e0 * e1, kk).astype(np.complex128)
    B = np.transpose(net.leaves[1], [lb.index(x) for x in (2, 3, 4)]).reshape(e2 * e3, kk).astype(np.complex128)
    exact = (A @ B.T).reshape(e0, e1, e2, e3)
    bound = (3 * 2.0 ** -16 * ((np.abs(A.real) + np.abs(A.imag)) @ (np.abs(B.real) + np.abs(B.imag)).T)
             .reshape(e0, e1, e2, e3))
    if order != "natural":
        exact = exact.transpose(0, 2, 1, 3)
        bound = bound.transpose(0, 2, 1, 3)
    assert np.all(np.abs(np.asarray(z) - exact) <= bound + 1e-6 * np.abs(exact))
    print(f"presplit bf16x3 {order} {leaves}: err vs emulation {err:.2e}, bitwise = wide tile", flush=True)


PRESPLIT_3M_CASES = {
    # extents, stored labels of A and of B
    "even_k": ([64, 65, 66, 64, 200], (0, 1, 4), (2, 3, 4)),
    "odd_k": ([64, 65, 66, 64, 201], (0, 1, 4), (2, 3, 4)),
    "permuted": ([64, 65, 64, 66, 1024], (4, 1, 0), (4, 3, 2)),
    "permuted_odd": ([66, 63, 63, 66, 1024], (4, 0, 1), (4, 3, 2)),
    "odd_n": ([64, 65, 65, 65, 256], (0, 1, 4), (2, 3, 4)),   # n = 4225: T rows end in a padding column
}


@pytest.mark.parametrize("case", list(PRESPLIT_3M_CASES))
@pytest.mark.parametrize("order", ["natural", "interleaved"])
def test_presplit_bf16x3_3m_is_bitwise_the_3m_tiles(ctx, order, case):
    """Split precision in the 3M form on pre-split planes: one GEMM of
    4160 x 4224 x k (ragged against the tile; odd k pads the last real k
    pair) splits A and B once into their r, i and s planes, runs the three
    real products on the pre-split kernel and combines them with the step's
    store (row-major or interleaved).  With permuted leaves (k = 1024, over
    the leaf cache's size) the leaf permutes write the planes themselves:
    "permuted" through the 16-byte pair kernel, "permuted_odd" (input runs
    of 63) through the element-wise one.  The result is bitwise that of the
    3M split tiles (variants 0 and 2 forced, leaves permuted to complex64 as
    usual) and of its hipGraph replays, within 1e-5 of the oracle's 3M split
    emulation, and every element within twice the split bound of the exact
    product."""
    ext, la, lb = PRESPLIT_3M_CASES[case]
    kk = ext[4]
    rng = np.random.Generator(np.random.PCG64(4161 + kk))
    ext = np.array(ext, dtype=np.int64)

    def cn(lab):
        shape = tuple(int(ext[l]) for l in lab)
        x = rng.standard_normal(shape + (2,), dtype=np.float32) * np.float32(np.sqrt(0.5))
        return x.view(np.complex64).reshape(shape)
    out = (0, 1, 2, 3) if order == "natural" else (0, 2, 1, 3)
    net = Network([cn(la), cn(lb)], [la, lb], ext, out)
    path = Path(np.array([[0, 1]], dtype=np.int32), ())
    print(f"presplit bf16x3 3M {order} {case}", flush=True)
    z, plan, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3, form=tnc.GEMM_3M)
    st = tnc.tnc_plan_get_step(plan.handle, 0)
    permuted = case.startswith("permuted")
    assert st.kernel == 0 and st.presplit == 1 and st.split == 1
    assert st.presplit_fused == (3 if permuted else 0)      # both permutes write planes
    assert plan.info.n_permutes == (2 if permuted else 0)
    assert st.natural == (1 if order == "natural" else 0)
    for v in (0, 2):
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, v)
        try:
            w, _, _ = run(ctx, net, path, prec=tnc.PREC_BF16X3, form=tnc.GEMM_3M)
        finally:
            tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)
        assert np.array_equal(np.asarray(z).view(np.uint64), np.asarray(w).view(np.uint64)), v
    tnc.tnc_plan_set_graph(plan.handle, True)
    for _ in range(2):
        g = plan.contract().reshape(np.asarray(z).shape)
        assert np.array_equal(g.view(np.uint64), np.asarray(z).view(np.uint64))
    emu = oc.contract(net, path, step=osp.split_step_3m)
    err = assert_close(z, emu, tol=1e-5, what="3M presplit vs emulation")
    e0, e1, e2, e3, _ = (int(x) for x in ext)
    A = np.transpose(net.leaves[0], [la.index(x) for x in (0, 1, 4)]).reshape(e0 * e1, kk).astype(np.complex128)
    B = np.transpose(net.leaves[1], [lb.index(x) for x in (2, 3, 4)]).reshape(e2 * e3, kk).astype(np.complex128)
    exact = (A @ B.T).reshape(e0, e1, e2, e3)
    bound = (2 * 3 * 2.0 ** -16 * ((np.abs(A.real) + np.abs(A.imag)) @ (np.abs(B.real) + np.abs(B.imag)).T)
             .reshape(e0, e1, e2, e3))
    if order != "natural":
        exact = exact.transpose(0, 2, 1, 3)
        bound = bound.transpose(0, 2, 1, 3)
    assert np.all(np.abs(np.asarray(z) - exact) <= bound + 1e-6 * np.abs(exact))
    print(f"presplit bf16x3 3M {order} {case}: err vs emulation {err:.2e}, bitwise = 3M tiles", flush=True)


def interleaved_pair(z, a, b, c, d, k, seed):
    """One contraction A[z, a, b, k] B[z, c, d, k] whose result order
    (z, a, c, b, d) interleaves the M labels (a, b) with the N labels (c, d):
    the GEMM stores it through the permuted-store epilogue."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = np.array([z, a, b, c, d, k], dtype=np.int64)
    la, lb = (0, 1, 2, 5), (0, 3, 4, 5)

    def cn(lab):
        shape = tuple(int(ext[l]) for l in lab)
        x = rng.standard_normal(shape + (2,), dtype=np.float32) * np.float32(np.sqrt(0.5))
        return x.view(np.complex64).reshape(shape)
    net = Network([cn(la), cn(lb)], [la, lb], ext, (0, 1, 3, 2, 4))
    return net, Path(np.array([[0, 1]], dtype=np.int32), ())


@pytest.mark.parametrize("kind", ["4M", "3M", "bf16x3", "bf16x3_3M"])
def test_every_tile_variant_through_the_permuted_store(ctx, kind):
    """Each of the seven MFMA workgroup shapes forced on a step stored in
    consumer order (per-row and per-column offset tables), on a ragged shape
    (m = 300, n = 105, k = 130, batch 3) and an interior one (m = 256,
    n = 128, k = 240, batch 2; no split-K: the GEMM stores), against the oracle: complex64 forms within
    1e-5 (and elementwise), split-bf16x3 (4M and 3M forms) within 1e-5 of
    its emulation and within its a-priori bound of the exact result."""
    prec = tnc.PREC_BF16X3 if kind.startswith("bf16x3") else tnc.PREC_C64
    form = tnc.GEMM_3M if kind.endswith("3M") else tnc.GEMM_4M
    cases = [interleaved_pair(3, 12, 25, 7, 15, 130, seed=41), interleaved_pair(2, 16, 16, 8, 16, 240, seed=42)]
    refs = [oc.contract(net, path) for net, path in cases]
    emu_step = {"bf16x3": osp.split_step, "bf16x3_3M": osp.split_step_3m}.get(kind)
    emus = [oc.contract(net, path, step=emu_step) for net, path in cases] if emu_step else None
    for variant in range(tnc.tnc_gemm_variant_count()):
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, variant)
        try:
            for q, (net, path) in enumerate(cases):
                print(f"permuted store, variant {variant} {kind} case {q}", flush=True)
                got, plan, tn = run(ctx, net, path, prec=prec, form=form)
                st = plan.step(0)
                assert st.kernel == 0 and st.natural == 0 and st.split == 1, (st.kernel, st.natural, st.split)
                if emus:
                    assert_close(got, emus[q], what=f"variant {variant} case {q} vs emulation")
                    assert_close(got, refs[q], tol=max(1e-5, 8 * 2.0 ** -16), what=f"variant {variant} case {q}")
                else:
                    assert_close(got, refs[q], what=f"variant {variant} case {q}")
                plan.close()
                tn.close()
        finally:
            tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)


def test_pair_permuted_operands(ctx):
    net, path = pair_network(10, 9, 8, seed=3)
    print("pair 10/9/8", flush=True)
    got, plan, _ = run(ctx, net, path)
    assert plan.info.n_permutes == 2
    ref = oc.contract(net, path)
    assert_close(got, ref)


def test_pair_batch(ctx):
    net, path = pair_network(8, 7, 6, seed=4, batch=8)
    print("pair batch", flush=True)
    got, plan, _ = run(ctx, net, path)
    assert plan.step(0).h == 8
    assert_close(got, oc.contract(net, path))


def test_direct_device_output_single_contraction(ctx):
    net, path = pair_network(9, 8, 7, seed=5)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    out = torch.empty(plan.info.n_result, dtype=torch.complex64, device="cuda")
    tnc.tnc_contract_async(plan.handle, 0, 1, out.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    ref = oc.contract(net, path)
    assert_close(out.cpu().numpy().reshape(ref.shape), ref)


def test_async_outputs_and_context_sync(ctx):
    """tnc_contract_async into a complex128 device buffer (FP64 sum over a
    sliced range) and into complex64, completed by tnc_ctx_sync alone: equal
    to the synchronous result (bitwise for complex128, its rounding for
    complex64)."""
    net, path = configs.circuit12(open_qubits=(0, 5))
    sl = greedy_slice(net, path.pairs, n_sliced=2)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, sl)
    want = plan.contract()
    n = plan.info.n_result
    out128 = torch.empty(n, dtype=torch.complex128, device="cuda")
    out64 = torch.empty(n, dtype=torch.complex64, device="cuda")
    tnc.tnc_contract_async(plan.handle, 0, plan.info.n_slices, out128.data_ptr(), tnc.OUT_C128)
    tnc.tnc_ctx_sync(ctx.handle)
    got128 = out128.cpu().numpy()
    tnc.tnc_contract_async(plan.handle, 0, plan.info.n_slices, out64.data_ptr(), tnc.OUT_C64)
    tnc.tnc_ctx_sync(ctx.handle)
    got64 = out64.cpu().numpy()
    assert np.array_equal(got128.view(np.uint64), np.asarray(want).view(np.uint64))
    assert np.array_equal(got64, np.asarray(want).astype(np.complex64))


def test_degenerate_networks(ctx):
    rng = np.random.Generator(np.random.PCG64(8))
    # one leaf, no steps, result in a permuted order
    x = (rng.standard_normal((2, 3, 4)) + 1j * rng.standard_normal((2, 3, 4))).astype(np.complex64)
    net = Network([x], [(0, 1, 2)], np.array([2, 3, 4]), (2, 0, 1))
    got, _, _ = run(ctx, net, Path(np.zeros((0, 2), dtype=np.int32)))
    assert np.array_equal(got, np.transpose(x, (2, 0, 1)).astype(np.complex128))
    # outer product (no shared label, k = 1) and an extent-1 label
    a = (rng.standard_normal((5, 1)) + 0j).astype(np.complex64)
    b = (rng.standard_normal((1, 7)) + 0j).astype(np.complex64)
    c = (rng.standard_normal((3,)) + 0j).astype(np.complex64)
    net = Network([a, b, c], [(0, 1), (1, 2), (3,)], np.array([5, 1, 7, 3]), (3, 2, 0))
    path = Path(np.array([[0, 1], [3, 2]], dtype=np.int32))
    got, _, _ = run(ctx, net, path)
    assert_close(got, oc.contract(net, path), tol=1e-6)
    # closed scalar network of two vectors
    u = (rng.standard_normal(6) + 1j * rng.standard_normal(6)).astype(np.complex64)
    v = (rng.standard_normal(6) + 1j * rng.standard_normal(6)).astype(np.complex64)
    net = Network([u, v], [(0,), (0,)], np.array([6]), ())
    got, _, _ = run(ctx, net, Path(np.array([[0, 1]], dtype=np.int32)))
    ref = complex(np.sum(u.astype(np.complex128) * v.astype(np.complex128)))
    assert abs(got - ref) <= 1e-6 * abs(ref)


def test_device_errors_are_status_codes(ctx):
    net, path = configs.circuit12()
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_contract(plan.handle, 0, 2, 1)      # only one slice exists
    assert e.value.status == tnc.E_ARG
    small = tnc.Context(0, arena_bytes=4096)
    tn2 = tnc.Network(small, net.labels, net.extents, net.open, net.c64().leaves)
    with pytest.raises(tnc.TncError) as e:
        tnc.Plan(tn2, path.pairs)
    assert e.value.status == tnc.E_NOMEM
    # the context still works afterwards
    assert abs(plan.contract()[0]) > 0


def test_graph_replay_matches_eager(ctx):
    """Chunks replayed as captured hipGraphs give bitwise the eager result,
    replay after replay, with other eager work on the stream in between."""
    net, path = configs.circuit12()
    sl = greedy_slice(net, path.pairs, n_sliced=4)
    p = Path(path.pairs, sl)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    eager = tnc.Plan(tn, p.pairs, p.sliced)
    tnc.tnc_plan_set_max_chunk(eager.handle, 4)
    graph = tnc.Plan(tn, p.pairs, p.sliced)
    tnc.tnc_plan_set_max_chunk(graph.handle, 4)
    tnc.tnc_plan_set_graph(graph.handle, True)
    ref = eager.contract()
    other_net, other_path = configs.grid8(4, 4, 3)
    other = tnc.Plan(tnc.Network(ctx, other_net.labels, other_net.extents, other_net.open,
                                 other_net.c64().leaves), other_path.pairs)
    for rep in range(4):
        got = graph.contract()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), rep
        other.contract()                          # eager work between replays
        part = graph.contract(3, 9)               # partial range: other chunk plans, same graphs
        assert np.array_equal(part.view(np.uint64), eager.contract(3, 9).view(np.uint64)), rep
    # single-slice direct device output through a graph
    net2, path2 = pair_network(9, 8, 7, seed=6)
    tn2 = tnc.Network(ctx, net2.labels, net2.extents, net2.open, net2.c64().leaves)
    pe, pg = tnc.Plan(tn2, path2.pairs), tnc.Plan(tn2, path2.pairs)
    tnc.tnc_plan_set_graph(pg.handle, True)
    oe = torch.empty(pe.info.n_result, dtype=torch.complex64, device="cuda")
    og = torch.empty_like(oe)
    tnc.tnc_contract_async(pe.handle, 0, 1, oe.data_ptr(), tnc.OUT_C64)
    for _ in range(3):
        og.zero_()
        tnc.tnc_contract_async(pg.handle, 0, 1, og.data_ptr(), tnc.OUT_C64)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(oe), torch.view_as_real(og))


def test_graph_cache_cap_falls_back_to_eager(ctx):
    """Every new output buffer of a single-slice direct-output run is a new
    graph key; past the per-plan cap (64 graphs) runs are launched eagerly.
    80 distinct buffers, then the first ones again: all bitwise equal to the
    eager plan's result."""
    net, path = pair_network(8, 7, 6, seed=11)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    pe, pg = tnc.Plan(tn, path.pairs), tnc.Plan(tn, path.pairs)
    tnc.tnc_plan_set_graph(pg.handle, True)
    n = pe.info.n_result
    ref = torch.empty(n, dtype=torch.complex64, device="cuda")
    tnc.tnc_contract_async(pe.handle, 0, 1, ref.data_ptr(), tnc.OUT_C64)
    outs = [torch.zeros(n, dtype=torch.complex64, device="cuda") for _ in range(80)]
    for o in outs + outs[:8]:
        o.zero_()
        tnc.tnc_contract_async(pg.handle, 0, 1, o.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert torch.equal(torch.view_as_real(o), torch.view_as_real(ref)), i
    pg.close()
    pe.close()
    tn.close()


def _bits(x):
    return np.asarray(x).view(np.uint64)


@pytest.mark.parametrize("case", ["circuit12_sliced", "circuit12_all", "grid8_bf16x3", "circuit16_wide"])
def test_level_grouping_is_bitwise_step_order(ctx, case):
    """Level-grouped launches (one launch per tree level for the small GEMMs
    and plain leaf gathers) give bitwise the step-by-step result, eagerly and
    replayed from captured graphs, also on chunks whose leaves carry fixed
    sliced labels (per-chunk base offsets)."""
    prec = tnc.PREC_C64
    max_chunk = None
    if case == "circuit12_sliced":
        net, path = configs.circuit12()
        sl = greedy_slice(net, path.pairs, n_sliced=4)
        path = Path(path.pairs, sl)
        max_chunk = 4
    elif case == "circuit12_all":
        circ = configs.circuit12_circuit()
        net = circuit_network(circ, open_qubits=range(12))
        path = greedy_path(net)
    elif case == "grid8_bf16x3":
        net, _ = prescaled_grid(8, 8, 4, seed=1002)
        path = greedy_path(net)
        prec = tnc.PREC_BF16X3
    else:
        circ = random_circuit(4, 4, 10, seed=77)
        net = circuit_network(circ, open_qubits=range(4))
        path = greedy_path(net)
    print("grouping", case, flush=True)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plans = {}
    for grouping in (0, 1):
        for graph in (0, 1):
            p = tnc.Plan(tn, path.pairs, path.sliced, prec)
            tnc.tnc_plan_set_grouping(p.handle, grouping)
            if max_chunk:
                tnc.tnc_plan_set_max_chunk(p.handle, max_chunk)
            tnc.tnc_plan_set_graph(p.handle, graph)
            plans[grouping, graph] = p
    ref = plans[0, 0].contract()
    for key, p in plans.items():
        for rep in range(2):
            got = p.contract()
            assert np.array_equal(_bits(got), _bits(ref)), (key, rep)
    # the grouped plan really groups: one small-GEMM launch per level at most
    g = plans[1, 0]
    tnc.tnc_plan_set_profile(g.handle, True)
    g.contract()
    ms, launches = tnc.tnc_plan_get_profile(g.handle, -3)
    n_small = sum(1 for s in range(g.info.n_steps) if g.step(s).kernel == 1)
    print(f"{case}: {n_small} small steps in {launches} grouped launches", flush=True)
    if n_small > 1:
        assert 1 <= launches < n_small
    ref_or = complex(oc.contract(net, path)) if not net.open else None
    if ref_or is not None and prec == tnc.PREC_C64:
        z = complex(ref[0])
        assert abs(z - ref_or) <= 1e-5 * abs(ref_or)


@pytest.mark.parametrize("dims, batch", [((7, 16, 6), 1), ((2, 20, 1), 1), ((3, 10, 9), 64), ((5, 12, 3), 4)],
                         ids=["splitk_mfma", "splitk_dot", "transposed", "skinny_split"])
@pytest.mark.parametrize("prec, form", [(tnc.PREC_C64, tnc.GEMM_4M), (tnc.PREC_C64, tnc.GEMM_3M),
                                        (tnc.PREC_BF16X3, tnc.GEMM_4M)], ids=["4M", "3M", "bf16x3"])
def test_split_k_and_transposed_launches(ctx, dims, batch, prec, form):
    """Steps run with K split into parts (partials summed by the split-K
    epilogue), or transposed so that MFMA tiles fill, match the oracle."""
    net, path = pair_network(*dims, seed=8, batch=batch)
    print("launch shapes", dims, batch, prec, form, flush=True)
    got, plan, _ = run(ctx, net, path, prec=prec, form=form)
    s = plan.step(0)
    ref = oc.contract(net, path)
    err = rel_fro(got, ref)
    print(f"h {s.h} m {s.m} n {s.n} k {s.k}: kernel {s.kernel} swapped {s.swapped} split {s.split}; "
          f"err {err:.2e}", flush=True)
    if prec == tnc.PREC_BF16X3:
        emu = oc.contract(net, path, step=osp.split_step)
        assert_close(got, emu)
        assert_close(got, ref, tol=max(1e-5, 4 * 2.0 ** -16))
    else:
        assert_close(got, ref)


def test_replaced_leaves_reach_cached_copies(ctx):
    """Leaves are permuted once into the plan's cache; replacing one (host or
    device copy) refreshes the cached copy before the next run, eager and
    from a captured graph."""
    from workloads.circuits import haar_unitary
    circ = configs.circuit12_circuit()
    net = circuit_network(circ)
    path = greedy_path(net)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    eager = tnc.Plan(tn, path.pairs)
    graph = tnc.Plan(tn, path.pairs)
    tnc.tnc_plan_set_graph(graph.handle, True)
    assert eager.info.n_cached_leaves > 0
    rng = np.random.Generator(np.random.PCG64(31))
    two_q = [g for g, (qs, _) in enumerate(circ.gates) if len(qs) == 2]
    gates = list(circ.gates)
    for rep, how in enumerate(("initial", "host", "device", "host")):
        if how != "initial":
            g = two_q[int(rng.integers(0, len(two_q)))]
            u = haar_unitary(rng, 4)
            gates[g] = (gates[g][0], u)
            t = circ.n_qubits + g                      # leaf of gate g
            vals = np.ascontiguousarray(u.reshape(2, 2, 2, 2)).astype(np.complex64)
            if how == "host":
                tnc.tnc_net_set_tensor(tn.handle, t, vals)
            else:
                dev = torch.from_numpy(vals.reshape(-1)).cuda()
                tnc.tnc_net_set_tensor_device(tn.handle, t, dev.data_ptr())
                torch.cuda.synchronize()
        sv = osv.amplitude(circ.n_qubits, [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in gates],
                           circ.bitstring)
        for p in (eager, graph):
            z = complex(p.contract()[0])
            print(f"{how}: {abs(z - sv) / abs(sv):.2e}", flush=True)
            assert abs(z - sv) <= 1e-5 * abs(sv), (rep, how)


def test_batched_bitstring_amplitudes(ctx):
    """64 amplitude queries of one circuit as one network (a batch label on
    the projector leaves): every step that sees a projector runs batched
    over the 64 bitstrings in one launch; each amplitude matches the state
    vector and the single-bitstring plan."""
    from workloads.circuits import circuit_network_batched
    circ = configs.circuit12_circuit()
    rng = np.random.Generator(np.random.PCG64(64))
    bits = rng.integers(0, 2, size=(64, circ.n_qubits))
    net = circuit_network_batched(circ, bits)
    path = greedy_path(net)
    print("batched bitstrings", flush=True)
    z, plan, _ = run(ctx, net, path)
    gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
    sv = osv.run(circ.n_qubits, gates)
    ref = np.array([sv[tuple(b)] for b in bits])
    assert z.shape == (64,)
    err = np.max(np.abs(z - ref)) / np.max(np.abs(ref))
    print(f"64 amplitudes: max err / max |amp| {err:.2e}, steps with batch {sum(plan.step(s).h > 1 for s in range(plan.info.n_steps))}", flush=True)
    assert rel_fro(z, ref) <= 1e-5 and err <= 1e-5
    single = circuit_network(circ, bitstring=bits[5])
    z5, _, _ = run(ctx, single, greedy_path(single))
    assert abs(z[5] - z5) <= 1e-5 * abs(z5)


@pytest.mark.parametrize("seed", range(6))
def test_random_trees_odd_extents_and_slices(ctx, seed):
    """Random tree networks with extents 1..5 (non-power-of-two batch and
    slice extents, extent-1 labels, a rank-0 leaf), two sliced labels and
    every chunk size: each matches the oracle; chunking does not change the
    sum beyond FP64 rounding."""
    rng = np.random.Generator(np.random.PCG64(4100 + seed))
    n_leaves = int(rng.integers(5, 12))
    labels = [[] for _ in range(n_leaves)]
    nxt = 0
    for t in range(1, n_leaves):
        s = int(rng.integers(0, t))
        labels[s].append(nxt); labels[t].append(nxt); nxt += 1
    for _ in range(n_leaves // 2):
        s, t = rng.choice(n_leaves, 2, replace=False)
        labels[int(s)].append(nxt); labels[int(t)].append(nxt); nxt += 1
    opn = []
    for _ in range(2):
        t = int(rng.integers(0, n_leaves))
        labels[t].append(nxt); opn.append(nxt); nxt += 1
    labels.append([])                                    # a rank-0 leaf (a scalar factor)
    ext = rng.integers(1, 6, size=nxt).astype(np.int64)
    labels = [tuple(int(x) for x in rng.permutation(l)) for l in labels]
    leaves = [(rng.standard_normal(tuple(int(ext[l]) for l in lab) or ()) +
               1j * rng.standard_normal(tuple(int(ext[l]) for l in lab) or ())).astype(np.complex128)
              for lab in labels]
    net = Network(leaves, labels, ext, tuple(opn))
    path = greedy_path(net)
    closed = [l for l in range(nxt) if l not in opn and ext[l] > 1]
    sl = tuple(int(x) for x in rng.choice(closed, size=min(2, len(closed)), replace=False))
    p = Path(path.pairs, sl)
    ref = oc.contract(net, p)
    print(f"random tree seed {seed}: {n_leaves + 1} leaves, sliced {sl} extents {[int(ext[l]) for l in sl]}",
          flush=True)
    n_slices = int(np.prod([ext[l] for l in sl])) if sl else 1
    vals = []
    for mc in sorted({1, int(ext[sl[-1]]) if sl else 1, n_slices}):
        got, plan, _ = run(ctx, net, p, max_chunk=mc)
        assert_close(np.asarray(got), np.asarray(ref), what=str(mc))
        vals.append(np.asarray(got))
    for v in vals[1:]:
        assert rel_fro(v, vals[0]) <= 1e-12


def test_profile_counts_survive_long_sessions(ctx):
    """A profiled plan run 20,000 times (its MFMA step's launches timed with
    events, past the point where finished timings are folded without
    waiting) reports every launch."""
    net, path = pair_network(9, 8, 7, seed=12)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    tnc.tnc_plan_set_profile(plan.handle, True)
    out = torch.empty(plan.info.n_result, dtype=torch.complex64, device="cuda")
    tnc.tnc_contract_async(plan.handle, 0, 1, out.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    _, per_run = tnc.tnc_plan_get_profile(plan.handle, 0)
    assert per_run >= 1
    n_runs = 20000
    for _ in range(n_runs):
        tnc.tnc_contract_async(plan.handle, 0, 1, out.data_ptr(), tnc.OUT_C64)
    torch.cuda.synchronize()
    ms, launches = tnc.tnc_plan_get_profile(plan.handle, 0)
    assert launches == per_run * (n_runs + 1) and ms > 0
    plan.close()
    tn.close()


@pytest.mark.parametrize("case", ["circuit12_grouped", "circuit12_stepwise", "grid8_4M", "grid8_3M",
                                  "grid8_bf16x3", "interleaved_pair", "sliced_circuit20"])
def test_separate_transpose_store_is_bitwise_the_epilogue(ctx, case):
    """Store order 1 (the GEMM stores in launch order, a separate transpose
    writes the consumer's order) gives bitwise the results of the
    permuted-store epilogue (store order 0): the same products, moved by a
    bit copy instead of the epilogue's addressing."""
    prec, form, grouping, sl = tnc.PREC_C64, tnc.GEMM_4M, True, ()
    if case.startswith("circuit12"):
        net, path = configs.circuit12(open_qubits=(0, 5, 11))
        grouping = case.endswith("grouped")
    elif case.startswith("grid8"):
        net, _ = prescaled_grid(8, 8, 4, seed=1002)
        path = greedy_path(net)
        prec = tnc.PREC_BF16X3 if case.endswith("bf16x3") else tnc.PREC_C64
        form = tnc.GEMM_3M if case.endswith("3M") else tnc.GEMM_4M
    elif case == "interleaved_pair":
        net, path = interleaved_pair(3, 12, 25, 7, 15, 130, seed=43)
    else:
        circ = random_circuit(4, 5, 10, seed=4321)
        net = circuit_network(circ)
        p = greedy_path(net)
        sl = greedy_slice(net, p.pairs, n_sliced=3)
        path = Path(p.pairs, sl)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    got = {}
    for mode in (0, 1):
        plan = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
        tnc.tnc_plan_set_grouping(plan.handle, grouping)
        tnc.tnc_plan_set_store_order(plan.handle, mode)
        if sl:
            tnc.tnc_plan_set_max_chunk(plan.handle, 4)
        got[mode] = plan.contract()
        n_perm = tnc.tnc_plan_get_info(plan.handle).n_permuted_stores
        plan.close()
    print(f"{case}: {n_perm} permuted-store steps", flush=True)
    assert n_perm > 0
    assert np.array_equal(got[0].view(np.uint64), got[1].view(np.uint64))
    ref = oc.contract(net, path)
    if prec == tnc.PREC_C64:
        assert_close(got[1], np.asarray(ref).reshape(-1))
    tn.close()


@pytest.mark.parametrize("prec", [tnc.PREC_C64, tnc.PREC_BF16X3], ids=["c64", "bf16x3"])
def test_sliced_leaves_read_in_place(ctx, prec):
    """Leaves whose sliced labels are fixed per chunk are read in place by
    the one-thread-per-output GEMMs that consume them (row and K offset
    tables, the chunk's base offset on the device) instead of being gathered
    into the arena before every batch: the results match the oracle and are
    bitwise the same level-grouped and step by step, eager and replayed."""
    circ = random_circuit(4, 5, 9, seed=5151)
    net = circuit_network(circ)
    p = greedy_path(net)
    sl = greedy_slice(net, p.pairs, n_sliced=4)
    path = Path(p.pairs, sl)
    ref = complex(oc.contract(net, path))
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    got = {}
    for grouping in (True, False):
        for graph in (False, True):
            for cap in (1, 4):
                plan = tnc.Plan(tn, path.pairs, path.sliced, prec)
                tnc.tnc_plan_set_grouping(plan.handle, grouping)
                tnc.tnc_plan_set_graph(plan.handle, graph)
                tnc.tnc_plan_set_max_chunk(plan.handle, cap)
                info = tnc.tnc_plan_get_info(plan.handle)
                assert info.n_inplace_leaves > 0
                z = plan.contract()
                z2 = plan.contract()                      # graph replay (or eager again)
                assert np.array_equal(z.view(np.uint64), z2.view(np.uint64))
                got[(grouping, graph, cap)] = z
                plan.close()
    print(f"in-place leaves: {info.n_inplace_leaves}", flush=True)
    for cap in (1, 4):
        base = got[(True, False, cap)]
        for key, z in got.items():
            if key[2] == cap:
                assert np.array_equal(z.view(np.uint64), base.view(np.uint64)), key
    tol = 1e-5 if prec == tnc.PREC_C64 else max(1e-5, 4 * 2.0 ** -16 * tree_depth(net.n_leaves, path.pairs))
    for z in got.values():
        assert abs(complex(z[0]) - ref) <= tol * abs(ref)
    tn.close()
