"""Host-side tests of the C ABI library (no GPU needed).

The library is loaded and every symbol the header declares must be exported.
Plans built on a host-only context are compared with the oracle's reordering
pass (paper Sec. IV-A) and cost model (Sec. II-B): orders and step groups are
integer data and must match exactly.
"""
import json
import os
import re

import numpy as np
import pytest

from oracle import costs as ocost
from oracle import reorder as orr
from paper_2606_01852_amd import tnc
from workloads import configs
from workloads.grids import random_grid_network
from workloads.network import Network
from workloads.paths import greedy_path, greedy_slice, random_greedy_path

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tnc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tnc.lib()
    names = header_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(tnc.exported_symbols()), set(names) ^ set(tnc.exported_symbols())
    assert "gfx950" in tnc.tnc_version()


def test_device_count_never_fails():
    n = tnc.tnc_device_count()
    assert isinstance(n, int) and n >= 0


@pytest.fixture(scope="module")
def hctx():
    return tnc.Context(-1)


def plan_for(hctx, net, path, sliced=()):
    tn = tnc.Network(hctx, net.labels, net.extents, net.open)
    return tn, tnc.Plan(tn, path.pairs, sliced)


def compare_with_oracle(plan, net, path, sliced=()):
    rm = set(sliced)
    labels = [tuple(l for l in lab if l not in rm) for lab in net.labels]
    target, steps = orr.reorder(labels, path.pairs, net.open)
    n_ids = net.n_leaves + len(path.pairs)
    for i in range(n_ids):
        assert plan.order(i) == target[i], i
    costs = ocost.step_costs(steps, target, net.extents)
    for s, (st, c) in enumerate(zip(steps, costs)):
        si = plan.step(s)
        assert (si.A, si.B, si.C) == (st["A"], st["B"], st["C"]), s
        assert (si.nH, si.nM, si.nN, si.nK) == tuple(len(st[g]) for g in "HMNK"), s
        assert (si.h, si.m, si.n, si.k) == (c["h"], c["m"], c["n"], c["k"]), s
        assert bool(si.natural) == st["natural"], s
    tot = ocost.path_totals(costs)
    assert plan.info.flops_per_slice == pytest.approx(tot["flops"], rel=1e-12)
    assert plan.info.bytes_per_slice == pytest.approx(8 * tot["Cm"], rel=1e-12)
    return target, steps


def test_fig3_example_through_the_library(hctx, golden_dir):
    d = json.load(open(os.path.join(golden_dir, "fig3_reorder.json")))
    L = d["labels"]
    lab = lambda s: tuple(L[c] for c in s)
    labels = [lab(d["leaves"][n]) for n in ("I1", "I2", "I3")]
    ids = {"I1": 0, "I2": 1, "I3": 2, "I4": 3, "I5": 4}
    pairs = np.array([[ids[a], ids[b]] for a, b in d["pairs"]], dtype=np.int32)
    tn = tnc.Network(hctx, labels, np.full(8, 2), lab(d["root_order"]))
    plan = tnc.Plan(tn, pairs)
    for name, want in d["expected"].items():
        assert tuple(plan.order(ids[name])) == lab(want), name
    assert plan.step(0).natural == 0 and plan.step(1).natural == 0
    assert plan.info.n_permuted_stores == 2


def _random_tree_network(rng, n_leaves, n_open):
    labels = [[] for _ in range(n_leaves)]
    nxt = 0
    for t in range(1, n_leaves):
        s = int(rng.integers(0, t))
        labels[s].append(nxt); labels[t].append(nxt); nxt += 1
    for _ in range(n_leaves):
        s, t = rng.choice(n_leaves, 2, replace=False)
        labels[s].append(nxt); labels[t].append(nxt); nxt += 1
    opn = []
    for _ in range(n_open):
        t = int(rng.integers(0, n_leaves))
        labels[t].append(nxt); opn.append(nxt); nxt += 1
    labels = [tuple(int(x) for x in rng.permutation(l)) for l in labels]
    ext = rng.integers(1, 4, size=nxt).astype(np.int64)
    return Network([None] * n_leaves, labels, ext, tuple(opn))


@pytest.mark.parametrize("seed", range(20))
def test_planner_matches_oracle_on_random_trees(hctx, seed):
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    net = _random_tree_network(rng, int(rng.integers(2, 24)), int(rng.integers(0, 5)))
    path = random_greedy_path(net, seed=seed)
    tn, plan = plan_for(hctx, net, path)
    compare_with_oracle(plan, net, path)


def test_planner_matches_oracle_on_workloads(hctx):
    net, path = configs.circuit12()
    tn, plan = plan_for(hctx, net, path)
    compare_with_oracle(plan, net, path)
    assert plan.info.n_steps == 153 and plan.info.n_result == 1
    g = random_grid_network(8, 8, 4, seed=1002)
    gp = greedy_path(g)
    tn2, plan2 = plan_for(hctx, g, gp)
    compare_with_oracle(plan2, g, gp)


def test_planner_with_slices_matches_sliced_oracle(hctx):
    net, path = configs.circuit12()
    sl = greedy_slice(net, path.pairs, n_sliced=3)
    tn, plan = plan_for(hctx, net, path, sl)
    compare_with_oracle(plan, net, path, sl)
    assert plan.info.n_slices == 8


def test_pair_batch_structure(hctx):
    net, path = configs.pair_batch(batch=64)
    tn, plan = plan_for(hctx, net, path)
    s = plan.step(0)
    assert (s.h, s.m, s.n, s.k) == (64, 1024, 256, 1024)
    assert s.natural == 1 and plan.info.n_permutes == 2
    assert plan.info.flops_per_slice == 8 * 64 * 1024 * 256 * 1024


def test_pair30_structure(hctx):
    net, path = configs.pair30.__wrapped__() if hasattr(configs.pair30, "__wrapped__") else (None, None)
    # structure only: labels without data (the 2^30 entries are not generated here)
    M, K, N = list(range(16)), list(range(16, 30)), list(range(30, 44))
    rng = np.random.Generator(np.random.PCG64(1))
    labels = [tuple(int(x) for x in rng.permutation(M + K)), tuple(int(x) for x in rng.permutation(N + K))]
    tn = tnc.Network(hctx, labels, np.full(44, 2), M + N)
    plan = tnc.Plan(tn, np.array([[0, 1]], dtype=np.int32))
    s = plan.step(0)
    assert (s.m, s.n, s.k) == (2 ** 16, 2 ** 14, 2 ** 14) and s.kernel == 0
    assert plan.order(0) == M + K and plan.order(1) == N + K
    assert plan.info.flops_per_slice == 8.0 * 2 ** 44
    assert plan.info.transpose_bytes == 16.0 * (2 ** 30 + 2 ** 28)


def test_presplit_steps_and_their_plane_buffer(hctx):
    """Split precision plans large single GEMMs (h = 1, launch m and n >=
    4096) on pre-split planes: the step says so, the other precisions and
    small or batched steps do not, and the planned peak grows by exactly the
    planes' bytes (A rows padded to 256, B' = 2 rows per complex column
    padded to 128 columns, k padded to 16, 8 bytes per padded element
    each)."""
    def one_gemm(m, n, k, h=1):
        ext = [h, m, n, k]
        net = Network([None, None], [(0, 1, 3), (0, 2, 3)], np.array(ext, dtype=np.int64), (0, 1, 2))
        tn = tnc.Network(hctx, net.labels, net.extents, net.open)
        return tn, {prec: tnc.Plan(tn, np.array([[0, 1]], dtype=np.int32), (), prec)
                    for prec in (tnc.PREC_C64, tnc.PREC_BF16X3)}
    align = 256
    for (m, n, k, h, expect) in ((4100, 4200, 1000, 1, True), (65536, 16384, 16384, 1, True),
                                 (4096, 2048, 512, 1, False), (4096, 4096, 512, 2, False)):
        tn, plans = one_gemm(m, n, k, h)
        st = {prec: p.step(0) for prec, p in plans.items()}
        assert st[tnc.PREC_C64].presplit == 0
        assert st[tnc.PREC_BF16X3].presplit == (1 if expect else 0), (m, n, k, h)
        grow = plans[tnc.PREC_BF16X3].info.peak_bytes - plans[tnc.PREC_C64].info.peak_bytes
        if expect:
            s = st[tnc.PREC_BF16X3]
            lm, ln = (s.n, s.m) if s.swapped else (s.m, s.n)   # the launch's rows and columns
            planes = (-(-lm // 256) * 256 + 2 * (-(-ln // 128) * 128)) * (-(-k // 16) * 16) * 8
            assert grow == -(-planes // align) * align, (m, n, k, grow, planes)
        else:
            assert grow == 0
        for p in plans.values():
            p.close()
        # the 3M form: the r, i and s planes of both operands (real k in
        # blocks of 32, B's real rows padded to 256) and the three float32
        # products of m x 2 ceil(n / 2), each part 256-byte aligned
        p3 = {prec: tnc.Plan(tn, np.array([[0, 1]], dtype=np.int32), (), prec, tnc.GEMM_3M)
              for prec in (tnc.PREC_C64, tnc.PREC_BF16X3)}
        s3 = p3[tnc.PREC_BF16X3].step(0)
        assert s3.presplit == (1 if expect else 0) and s3.presplit_fused == 0
        grow3 = p3[tnc.PREC_BF16X3].info.peak_bytes - p3[tnc.PREC_C64].info.peak_bytes
        if expect:
            lm, ln = (s3.n, s3.m) if s3.swapped else (s3.m, s3.n)
            up = lambda x, a: -(-x // a) * a
            nh, kp = up(ln, 2) // 2, up(up(k, 2) // 2, 16)
            mp, np_ = up(lm, 256), 2 * up(nh, 128)
            want = up(3 * mp * kp * 8, align) + up(3 * np_ * kp * 8, align) + up(3 * lm * 2 * nh * 4, align)
            assert grow3 == up(want, align), (m, n, k, grow3, want)
        else:
            assert grow3 == 0
        for p in p3.values():
            p.close()
        tn.close()


def test_permutes_write_planes_only_for_whole_blocks(hctx):
    """A pre-split step's permuted leaves (over the leaf cache's size) write
    its planes themselves when their rows are whole plane blocks: k a
    multiple of 16 in the 4M form (16 complex k per block), of 32 in the 3M
    form (32 real k per block); otherwise they permute to complex64 and the
    step splits them."""
    for kk, want4, want3 in ((1024, 3, 3), (1040, 3, 0), (1000, 0, 0)):
        ext = np.array([64, 65, 64, 66, kk], dtype=np.int64)
        tn = tnc.Network(hctx, [(4, 1, 0), (4, 3, 2)], ext, (0, 1, 2, 3))
        for form, want in ((tnc.GEMM_4M, want4), (tnc.GEMM_3M, want3)):
            p = tnc.Plan(tn, np.array([[0, 1]], dtype=np.int32), (), tnc.PREC_BF16X3, form)
            st = p.step(0)
            assert (st.presplit, st.presplit_fused, p.info.n_permutes) == (1, want, 2), (kk, form)
            p.close()
        tn.close()


def test_launch_counts_of_a_run(hctx):
    """n_launches counts the launches of one eager run: level grouping cuts
    them, a step-by-step run issues at least one per step plus the
    reduction."""
    net, path = configs.circuit12()
    tn = tnc.Network(hctx, net.labels, net.extents, net.open)
    counts = {}
    for grouping in (False, True):
        p = tnc.Plan(tn, path.pairs)
        tnc.tnc_plan_set_grouping(p.handle, grouping)
        counts[grouping] = tnc.tnc_plan_get_info(p.handle).n_launches
        p.close()
    assert counts[False] >= len(path.pairs) + 1
    assert counts[True] < counts[False] // 4, counts
    tn.close()


def test_errors_are_reported_not_raised_across_the_abi(hctx):
    with pytest.raises(tnc.TncError) as e:       # closed hyperedge
        tnc.Network(hctx, [(0, 1), (1, 2), (1, 3)], [2, 2, 2, 2], [0, 2, 3])
    assert e.value.status == tnc.E_ARG and "joins exactly two" in str(e.value)
    with pytest.raises(tnc.TncError) as e:       # dangling closed label
        tnc.Network(hctx, [(0, 1), (1,)], [2, 2], [])
    assert e.value.status == tnc.E_ARG
    tn = tnc.Network(hctx, [(0, 1), (1, 2), (2,)], [2, 2, 2], [0])
    with pytest.raises(tnc.TncError) as e:       # id consumed twice
        tnc.Plan(tn, np.array([[0, 1], [0, 2]]))
    assert e.value.status == tnc.E_PATH
    with pytest.raises(tnc.TncError) as e:       # not a full tree
        tnc.Plan(tn, np.array([[0, 1]]))
    assert e.value.status == tnc.E_PATH
    with pytest.raises(tnc.TncError) as e:       # slicing an open label
        tnc.Plan(tn, np.array([[0, 1], [3, 2]]), sliced=[0])
    assert e.value.status == tnc.E_ARG
    # a host-only context with a budget reports planned peaks above it
    small = tnc.Context(-1, arena_bytes=1024)
    net, path = configs.circuit12()
    tn2 = tnc.Network(small, net.labels, net.extents, net.open)
    with pytest.raises(tnc.TncError) as e:
        tnc.Plan(tn2, path.pairs)
    assert e.value.status == tnc.E_NOMEM
    assert tnc.lib().tnc_last_error().decode()


@pytest.mark.parametrize("grouping", [1, 0])
def test_memory_plan_and_chunking(hctx, grouping):
    net, path = configs.circuit40(n_sliced=16)
    tn = tnc.Network(tnc.Context(-1, arena_bytes=8 << 30), net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs, path.sliced)
    tnc.tnc_plan_set_grouping(plan.handle, grouping)
    info = tnc.tnc_plan_get_info(plan.handle)
    assert info.n_slices == 2 ** 16
    assert info.max_intermediate <= 2 ** 19
    # first-fit placement stays close to the live-bytes lower bound: at each
    # point of the execution order (a step, or a level of the tree when
    # levels run as groups) the intermediates produced and not yet consumed
    # must all be resident
    from workloads.paths import path_tensors
    tens, _ = path_tensors(net, path.pairs, path.sliced)
    size = [int(np.prod([net.extents[l] for l in t])) * 8 for t in tens]
    n = net.n_leaves
    ns = len(path.pairs)
    consumer = {}
    for s_, (a, b) in enumerate(path.pairs):
        consumer[int(a)] = consumer[int(b)] = s_
    lvl = [0] * (n + ns)
    for s_, (a, b) in enumerate(path.pairs):
        lvl[n + s_] = 1 + max(lvl[a], lvl[b])
    when = (lambda s_: lvl[n + s_]) if grouping else (lambda s_: s_)
    end = when(ns - 1) + 1
    # split-K partial products (S x the step's output) are live during their step
    scratch = []
    for q in range(ns):
        st = plan.step(q)
        scratch.append(8 * st.h * st.m * st.n * st.split if st.split > 1 else 0)
    lb = 0
    for t in range(end + 1):
        live = sum(size[n + q] for q in range(ns)
                   if when(q) <= t <= (when(consumer[n + q]) if n + q in consumer else end))
        live += sum(scratch[q] for q in range(ns) if when(q) == t)
        lb = max(lb, live)
    assert lb <= info.peak_bytes <= 1.5 * lb + (1 << 20)
    assert info.max_chunk >= 64 and info.chunk_peak_bytes <= 8 << 30


def test_grouping_keeps_the_plan_shape(hctx):
    net, path = configs.circuit12()
    tn = tnc.Network(hctx, net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs)
    steps = [plan.step(s) for s in range(plan.info.n_steps)]
    tnc.tnc_plan_set_grouping(plan.handle, 0)
    for s, st in enumerate(steps):
        other = plan.step(s)
        assert (other.m, other.n, other.k, other.h, other.kernel) == (st.m, st.n, st.k, st.h, st.kernel)
    with pytest.raises(tnc.TncError):
        tnc.tnc_plan_set_grouping(0, 1)


def test_host_only_server_queues_without_running_and_refuses_changes():
    """A host-only context with an arena size serves as a dry run: requests
    are admitted and complete with TNC_E_UNSUPPORTED, outputs untouched.
    While it serves, every call that would change what the workers read is
    refused with TNC_E_BUSY; after tnc_serve_stop they work again."""
    bare = tnc.Context(-1)
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_serve_start(bare.handle, 2, 8)       # no arena size to admit against
    assert e.value.status == tnc.E_ARG
    ctx = tnc.Context(-1, arena_bytes=1 << 30)
    net, path = configs.circuit12()
    tn = tnc.Network(ctx, net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs)
    tnc.tnc_serve_start(ctx.handle, 3, 64)
    refused = [lambda: tnc.tnc_plan_set_max_chunk(plan.handle, 1),
               lambda: tnc.tnc_plan_autotune(plan.handle),
               lambda: tnc.tnc_plan_set_graph(plan.handle, True),
               lambda: tnc.tnc_plan_set_grouping(plan.handle, False),
               lambda: tnc.tnc_plan_set_profile(plan.handle, True),
               lambda: tnc.tnc_ctx_set_gemm_variant(ctx.handle, 2),
               lambda: tnc.tnc_net_set_tensor(tn.handle, 0, net.c64().leaves[0]),
               lambda: tnc.tnc_net_set_tensor_device(tn.handle, 0, 1 << 20),
               lambda: tnc.tnc_contract(plan.handle, 0, 1, 1)]
    for call in refused:
        with pytest.raises(tnc.TncError) as e:
            call()
        assert e.value.status == tnc.E_BUSY
    outs = [np.zeros(1, dtype=np.complex128) for _ in range(16)]
    ids = [tnc.tnc_submit(ctx.handle, plan.handle, 0, 1, o) for o in outs]
    for rid in ids:
        with pytest.raises(tnc.TncError) as e:
            tnc.tnc_wait(ctx.handle, rid)
        assert e.value.status == tnc.E_UNSUPPORTED
    assert all(o[0] == 0 for o in outs)
    tnc.tnc_serve_stop(ctx.handle)
    tnc.tnc_plan_set_max_chunk(plan.handle, 1)       # allowed again
    tnc.tnc_plan_set_grouping(plan.handle, False)


def test_handles_can_be_destroyed_in_any_order():
    net, path = configs.circuit12()
    for order in ("ctx_first", "net_first", "plan_first"):
        ctx = tnc.tnc_ctx_create(-1)
        n = tnc.tnc_net_create(ctx, net.labels, net.extents, net.open, None)
        p = tnc.tnc_plan_create(n, path.pairs)
        if order == "ctx_first":
            tnc.tnc_ctx_destroy(ctx)
            tnc.tnc_net_destroy(n)
            assert tnc.tnc_plan_get_info(p).n_steps == 153   # still usable
            tnc.tnc_plan_destroy(p)
        elif order == "net_first":
            tnc.tnc_net_destroy(n)
            tnc.tnc_plan_destroy(p)
            tnc.tnc_ctx_destroy(ctx)
        else:
            tnc.tnc_plan_destroy(p)
            tnc.tnc_net_destroy(n)
            tnc.tnc_ctx_destroy(ctx)


def test_slice_invariant_work_runs_once_per_batch(hctx):
    """In a batch of c slices, a step pays for a batch label only if its
    operands' subtrees hold that label: slice-invariant subtrees are computed
    once per batch, not once per slice.  The executed FLOPs of the largest
    batch are recomputed here from the label sets alone."""
    net, path = configs.circuit40(n_sliced=16)
    tn = tnc.Network(tnc.Context(-1, arena_bytes=8 << 30), net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs, path.sliced)
    info = plan.info
    c = info.max_chunk
    j = int(round(np.log2(c)))
    assert 2 ** j == c and j >= 1
    batched = set(int(l) for l in path.sliced[len(path.sliced) - j:])
    from workloads.paths import path_tensors
    _, ops = path_tensors(net, path.pairs, path.sliced)
    n = net.n_leaves
    holds = [set(int(l) for l in lab) & batched for lab in net.labels]
    executed = 0
    for s, (a, b) in enumerate(path.pairs):
        holds.append(holds[a] | holds[b])
        mult = int(np.prod([net.extents[l] for l in holds[n + s]]))
        executed += 8 * ops[s] * mult
        bs = tnc.tnc_plan_get_batch_step(plan.handle, s)     # the batched step's own view
        assert bs.h == mult and (bs.m, bs.n, bs.k) == (plan.step(s).m, plan.step(s).n, plan.step(s).k), s
    assert info.chunk_flops == executed
    # per-slice accounting would be c times the per-slice count; hoisting saves
    per_slice = c * info.flops_per_slice
    print(f"batch of {c}: executed {executed:.3e} FLOP vs {per_slice:.3e} slice by slice")
    assert executed < per_slice


@pytest.mark.parametrize("dims, batch, kernel, swapped, split", [
    ((7, 16, 6), 1, 0, 0, 512),     # 128 x 64 output, k = 2^16: one tile, K cut 512 ways
    ((2, 20, 1), 1, 2, 0, 1024),    # 4 x 2 outputs, k = 2^20: long dot, K cut 1024 ways
    ((3, 10, 9), 64, 0, 1, 8),      # 64 x (8 x 512), k = 2^10: MFMA only transposed, 256 tiles: K cut 8 ways
    ((10, 9, 8), 1, 0, 0, 4),       # 32 tiles, k = 512: K cut 4 ways (parts of 128)
    ((12, 9, 10), 1, 0, 0, 1),      # 512 tiles of 128 x 64: no split
    ((2, 3, 2), 1, 1, 0, 1),        # tiny: one thread per output
    ((6, 6, 6), 1, 1, 0, 1),        # 64 x 64 x 64 (2^18 MACs, short K): one thread per output
    ((8, 7, 8), 1, 0, 0, 1),        # 256 x 256 x 128 (2^23 MACs): MFMA, K too short to split
])
def test_launch_shape_decisions(hctx, dims, batch, kernel, swapped, split):
    """Kernel, orientation and split-K choice per step shape (host rules)."""
    from workloads.pairs import pair_network
    net, path = pair_network(*dims, seed=7, batch=batch)
    tn = tnc.Network(hctx, net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs)
    s = plan.step(0)
    assert (s.kernel, s.swapped, s.split) == (kernel, swapped, split)
    assert (s.m, s.n, s.k) == (2 ** dims[0], 2 ** dims[2], 2 ** dims[1])   # logical view unchanged
    if split > 1:    # the partials sit in the arena next to the result
        assert plan.info.peak_bytes >= 8 * s.h * s.m * s.n * (split + 1)


def _batched_circuit(n_rows=16):
    from workloads.circuits import circuit_network_batched
    circ = configs.circuit12_circuit()
    bits = np.zeros((n_rows, circ.n_qubits), dtype=np.int64)
    return circuit_network_batched(circ, bits)


def test_batcher_validation_and_cache_exclusion(hctx):
    """A batcher needs its batch label open, leading the open list and
    outermost in every leaf that carries it; one batcher per network; its
    leaves leave the plan's leaf cache.  All decided on the host."""
    net = _batched_circuit()
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
    assert len(carriers) == 12 and all(net.labels[t][0] == beta for t in carriers)
    path = greedy_path(net)
    tn = tnc.Network(hctx, net.labels, net.extents, net.open)
    plan = tnc.Plan(tn, path.pairs)
    cached_before = tnc.tnc_plan_get_info(plan.handle).n_cached_leaves

    def err(label, leaves):
        with pytest.raises(tnc.TncError) as e:
            tnc.Batcher(plan, label, leaves)
        return e.value.status

    closed = next(l for l in range(len(net.extents)) if l not in net.open)
    assert err(closed, carriers) == tnc.E_ARG                 # not open
    assert err(beta, carriers[:-1]) == tnc.E_ARG              # a carrier left out
    assert err(beta, carriers + [carriers[0]]) == tnc.E_ARG   # listed twice
    other = next(t for t in range(net.n_leaves) if t not in carriers)
    assert err(beta, carriers + [other]) == tnc.E_ARG         # leaf without the label
    b = tnc.Batcher(plan, beta, carriers)
    assert err(beta, carriers) == tnc.E_BUSY                  # one batcher per network
    with pytest.raises(tnc.TncError) as e:                    # rows need a serving context
        tnc.tnc_submit_row(hctx.handle, b.handle, [np.eye(2)[0]] * len(carriers), np.zeros(1, np.complex128))
    assert e.value.status == tnc.E_ARG
    assert tnc.tnc_plan_get_info(plan.handle).n_result == 16
    assert tnc.tnc_plan_get_info(plan.handle).n_cached_leaves == cached_before  # projectors: stored as targeted
    b.close()
    tnc.Batcher(plan, beta, carriers).close()                # free again after destroy

    # the label must lead the open list and be the outermost stored mode
    perm_net = Network(net.leaves, [tuple(reversed(l)) if t in carriers else l
                                    for t, l in enumerate(net.labels)], net.extents, net.open)
    tn2 = tnc.Network(hctx, perm_net.labels, perm_net.extents, perm_net.open)
    plan2 = tnc.Plan(tn2, path.pairs)
    with pytest.raises(tnc.TncError) as e:
        tnc.Batcher(plan2, beta, carriers)
    assert e.value.status == tnc.E_ARG


def test_batcher_leaves_leave_the_leaf_cache(hctx):
    """A batch-labelled leaf stored (beta, j, i) is targeted (beta, i, j)
    (reduced modes ascending): without a batcher it is permuted once into the
    leaf cache; a batcher rewrites it before every run, so the re-planned
    chunk permutes it per run instead."""
    labels = [(2, 1, 0), (0, 1)]
    ext = np.array([3, 5, 4], dtype=np.int64)
    tn = tnc.Network(hctx, labels, ext, (2,))
    plan = tnc.Plan(tn, [(0, 1)])
    assert plan.order(0) == [2, 0, 1]
    assert tnc.tnc_plan_get_info(plan.handle).n_cached_leaves == 1
    b = tnc.Batcher(plan, 2, [0])
    assert tnc.tnc_plan_get_info(plan.handle).n_cached_leaves == 0
    assert tnc.tnc_plan_get_info(plan.handle).n_permutes == 1
    b.close()


def test_choice_arguments_are_checked_before_use(hctx):
    """Precision, GEMM form and element types cross the ABI as plain integers
    and are checked before anything else uses them; permute arguments are
    checked before any device work (a host-only context then refuses it)."""
    import ctypes as C
    L = tnc.lib()
    tn = tnc.Network(hctx, [(0, 1), (1, 2), (2, 0)], np.array([3, 4, 5], dtype=np.int64), ())
    pairs = np.array([0, 1, 3, 2], dtype=np.int32)
    pp = pairs.ctypes.data_as(C.POINTER(C.c_int32))
    out = C.c_void_p()
    for prec, form, want in ((9, tnc.GEMM_4M, tnc.E_ARG), (-1, tnc.GEMM_4M, tnc.E_ARG),
                             (tnc.PREC_C64, 2, tnc.E_ARG), (tnc.PREC_BF16X3, -3, tnc.E_ARG)):
        assert L.tnc_plan_create(tn.handle, 2, pp, 0, None, prec, form, C.byref(out)) == want
    for prec in (tnc.PREC_C64, tnc.PREC_BF16X3):   # both forms compose with both precisions
        assert L.tnc_plan_create(tn.handle, 2, pp, 0, None, prec, tnc.GEMM_3M, C.byref(out)) == tnc.OK
        assert L.tnc_plan_destroy(out) == tnc.OK
    ranks = np.array([1, 1], dtype=np.int32)
    labs = np.array([0, 0], dtype=np.int32)
    ext = np.array([2], dtype=np.int64)
    net = C.c_void_p()
    assert L.tnc_net_create(hctx.handle, 2, ranks.ctypes.data_as(C.POINTER(C.c_int32)),
                            labs.ctypes.data_as(C.POINTER(C.c_int32)), 1,
                            ext.ctypes.data_as(C.POINTER(C.c_int64)), 0, None, None, 7, C.byref(net)) == tnc.E_ARG
    buf = np.zeros(4, dtype=np.complex64)
    e3 = np.array([4, 5, 6], dtype=np.int64)
    huge = np.array([1 << 30, 1 << 30, 64], dtype=np.int64)
    perm = np.array([2, 0, 1], dtype=np.int32)
    dup = np.array([2, 2, 1], dtype=np.int32)

    def permute(e, p):
        return L.tnc_permute(hctx.handle, buf.ctypes.data, buf.ctypes.data, 3, e.ctypes.data_as(C.POINTER(C.c_int64)),
                             p.ctypes.data_as(C.POINTER(C.c_int32)))
    assert permute(e3, dup) == tnc.E_ARG
    assert permute(huge, perm) == tnc.E_ARG
    assert permute(e3, perm) == tnc.E_UNSUPPORTED
    tn.close()
