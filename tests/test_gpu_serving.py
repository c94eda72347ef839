"""Continuous-batching server (C ABI): results alone vs in a mix, admission
by planned memory, queue limits, and parity of served amplitudes with the
oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import contract as oc  # noqa: E402
from paper_2606_01852_amd import tnc  # noqa: E402
from workloads.circuits import circuit_network, random_circuit  # noqa: E402
from workloads.network import Path  # noqa: E402
from workloads.paths import greedy_path, greedy_slice  # noqa: E402


def request_pool(n):
    """Small synthetic mix: grid circuits of 12..30 qubits, 1..64 slices."""
    rng = np.random.Generator(np.random.PCG64(4242))
    pool = []
    for i in range(n):
        rows, cols = [(3, 4), (4, 5), (4, 6), (5, 6), (4, 4)][i % 5]
        depth = int(rng.integers(6, 11))
        circ = random_circuit(rows, cols, depth, seed=7000 + i)
        net = circuit_network(circ)
        path = greedy_path(net)
        n_sl = int(rng.integers(0, 4)) * 2
        sl = greedy_slice(net, path.pairs, n_sliced=n_sl) if n_sl else ()
        pool.append((net, Path(path.pairs, sl)))
    return pool


@pytest.fixture(scope="module")
def served():
    arena = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    ctx._arena = arena
    pool = request_pool(10)
    nets, plans = [], []
    for net, path in pool:
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        nets.append(tn)
        plans.append(tnc.Plan(tn, path.pairs, path.sliced))
    yield ctx, pool, nets, plans
    for p in plans:
        p.close()
    for n in nets:
        n.close()
    ctx.close()


def run_all(ctx, plans, order, max_inflight):
    tnc.tnc_serve_start(ctx.handle, max_inflight, 1024)
    outs, ids = {}, {}
    for i in order:
        outs[i] = np.zeros(1, dtype=np.complex128)
        ids[i] = tnc.tnc_submit(ctx.handle, plans[i].handle, 0, plans[i].info.n_slices, outs[i])
    lat = {i: tnc.tnc_wait(ctx.handle, ids[i]) for i in order}
    tnc.tnc_serve_stop(ctx.handle)
    return outs, lat


def test_alone_equals_mix_and_matches_oracle(served):
    ctx, pool, nets, plans = served
    order = list(range(len(plans)))
    alone = {}
    for i in order:                       # one request at a time
        o, _ = run_all(ctx, plans, [i], 1)
        alone[i] = o[i]
    rng = np.random.Generator(np.random.PCG64(5))
    mixed_order = [int(x) for x in rng.permutation(order)] * 3   # repeats overlap each other
    tnc.tnc_serve_start(ctx.handle, 6, 1024)
    outs, ids = [], []
    for i in mixed_order:
        out = np.zeros(1, dtype=np.complex128)
        outs.append((i, out))
        ids.append(tnc.tnc_submit(ctx.handle, plans[i].handle, 0, plans[i].info.n_slices, out))
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    for i, out in outs:
        assert np.array_equal(out.view(np.uint64), alone[i].view(np.uint64)), i   # bitwise
    for i in order[:4]:
        net, path = pool[i]
        ref = complex(oc.contract(net, path))
        z = complex(alone[i][0])
        assert abs(z - ref) <= 1e-5 * abs(ref), (i, abs(z - ref) / abs(ref))


def test_admission_by_memory_queues_instead_of_failing(served):
    _, pool, _, _ = served
    net, path = pool[3]
    # an arena that holds exactly one request at a time
    probe = tnc.Context(-1)
    tp = tnc.Network(probe, net.labels, net.extents, net.open)
    pp = tnc.Plan(tp, path.pairs, path.sliced)
    need = pp.info.chunk_peak_bytes + (1 << 20)
    arena = torch.empty(int(need * 1.5), dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, path.sliced)
    tnc.tnc_serve_start(ctx.handle, 4, 64)
    outs = [np.zeros(1, dtype=np.complex128) for _ in range(8)]
    ids = [tnc.tnc_submit(ctx.handle, plan.handle, 0, plan.info.n_slices, o) for o in outs]
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # a full queue is refused with TNC_E_BUSY (one slot, queue of one)
    tnc.tnc_serve_start(ctx.handle, 1, 1)
    accepted, busy = [], 0
    keep = [np.zeros(1, dtype=np.complex128) for _ in range(6)]   # outputs must outlive the requests
    for o in keep:
        try:
            accepted.append(tnc.tnc_submit(ctx.handle, plan.handle, 0, plan.info.n_slices, o))
        except tnc.TncError as e:
            assert e.status == tnc.E_BUSY
            busy += 1
    assert busy >= 1 and len(accepted) >= 1
    for rid in accepted:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    with pytest.raises(tnc.TncError) as e:     # no server any more
        tnc.tnc_submit(ctx.handle, plan.handle, 0, 1, np.zeros(1, dtype=np.complex128))
    assert e.value.status == tnc.E_ARG


def test_contract_is_refused_while_serving(served):
    ctx, _, _, plans = served
    tnc.tnc_serve_start(ctx.handle, 2, 16)
    with pytest.raises(tnc.TncError) as e:
        plans[0].contract()
    assert e.value.status == tnc.E_BUSY
    tnc.tnc_serve_stop(ctx.handle)
    assert plans[0].contract().shape == (1,)


def test_heavy_lane_keeps_results(served):
    """Heavy requests (planned work above a threshold) share a lane of few
    slots and light ones pass them in the queue; results stay bitwise those
    of one request at a time, whatever the lane setting."""
    ctx, pool, nets, plans = served
    order = list(range(len(plans)))
    work = [p.info.chunk_flops * (p.info.n_slices // p.info.max_chunk) for p in plans]
    threshold = float(np.median(work))
    print("planned work", [f"{w:.2e}" for w in work], "threshold", f"{threshold:.2e}", flush=True)
    alone = {}
    for i in order:
        o, _ = run_all(ctx, plans, [i], 1)
        alone[i] = o[i]
    with pytest.raises(tnc.TncError):            # no server running
        tnc.tnc_serve_set_heavy(ctx.handle, threshold, 1)
    rng = np.random.Generator(np.random.PCG64(6))
    mixed = [int(x) for x in rng.permutation(order)] * 2
    for heavy, slots in ((threshold, 1), (threshold, 2), (0.0, 1)):
        tnc.tnc_serve_start(ctx.handle, 6, 1024)
        with pytest.raises(tnc.TncError):
            tnc.tnc_serve_set_heavy(ctx.handle, heavy, 0)
        tnc.tnc_serve_set_heavy(ctx.handle, heavy, slots)
        outs, ids = [], []
        for i in mixed:
            out = np.zeros(1, dtype=np.complex128)
            outs.append((i, out))
            ids.append(tnc.tnc_submit(ctx.handle, plans[i].handle, 0, plans[i].info.n_slices, out))
        for rid in ids:
            tnc.tnc_wait(ctx.handle, rid)
        tnc.tnc_serve_stop(ctx.handle)
        for i, out in outs:
            assert np.array_equal(out.view(np.uint64), alone[i].view(np.uint64)), (heavy, slots, i)


def test_serving_pool_requests_match_the_state_vector():
    """Requests of the serving benchmark's own pool (the 20-qubit entries,
    1 to 1024 slices) served concurrently in complex64 and in split-bf16x3,
    against the brute-force state vector: 1e-5 for complex64, the split
    bound max(1e-5, 4 * 2^-16 * depth of the tree) for bf16x3."""
    from oracle import statevector as osv
    from workloads import configs
    arena = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    entries = [i for i in range(24) if np.prod(configs.serve_request_spec(i)[:2]) <= 20]
    assert len(entries) >= 3
    jobs = []
    for i in entries:
        circ, net, path, _ = configs.serve_request_circuit(i)
        gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
        ref = osv.amplitude(circ.n_qubits, gates, circ.bitstring)
        depth = [0] * net.n_leaves
        for a, b in path.pairs:
            depth.append(1 + max(depth[int(a)], depth[int(b)]))
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        for prec in (tnc.PREC_C64, tnc.PREC_BF16X3):
            plan = tnc.Plan(tn, path.pairs, path.sliced, prec)
            tol = 1e-5 if prec == tnc.PREC_C64 else max(1e-5, 4 * 2.0 ** -16 * depth[-1])
            jobs.append((i, prec, plan, tn, ref, tol, np.zeros(1, dtype=np.complex128)))
    tnc.tnc_serve_start(ctx.handle, 8, 256)
    ids = [tnc.tnc_submit(ctx.handle, j[2].handle, 0, j[2].info.n_slices, j[6]) for j in jobs]
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    for i, prec, plan, _, ref, tol, out in jobs:
        err = abs(complex(out[0]) - ref) / abs(ref)
        print(f"pool entry {i} ({plan.info.n_slices} slices, prec {prec}): err {err:.2e} (tol {tol:.1e})", flush=True)
        assert err <= tol, (i, prec)
    for j in jobs:
        j[2].close()
    ctx.close()


def _tree_depth(n_leaves, pairs):
    depth = [0] * n_leaves
    for a, b in pairs:
        depth.append(1 + max(depth[int(a)], depth[int(b)]))
    return depth[-1]


def test_serving_pool_requests_above_20_qubits():
    """Requests of the serving benchmark's pool beyond 20 qubits, served
    together in one mix:
      * a 24-qubit request (4 slices, complex64) against the brute-force
        state vector (1e-5);
      * two 25-qubit requests (64 slices; complex64 and split-bf16x3), whole
        sums against the FP64 tensor-network oracle;
      * a seeded sample of four pool entries of 28..48 qubits, three seeded
        slices each served as single-slice requests, against the FP64
        oracle's contraction of the same slice.  Per-slice amplitudes of
        random circuits are Porter-Thomas distributed, so each error is
        bounded relative to the root-mean-square of the request's sampled
        slices (the circuit40 reading); split-bf16x3 requests use their
        bound max(1e-5, 4 * 2^-16 * tree depth)."""
    from oracle import statevector as osv
    from workloads import configs
    from workloads.paths import path_cost
    arena = torch.empty(16 << 30, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    rng = np.random.Generator(np.random.PCG64(5005))
    big = [i for i in range(64) if np.prod(configs.serve_request_spec(i)[:2]) > 26
           and configs.serve_request_spec(i)[3] >= 3]
    sampled = []
    for i in rng.permutation(big):
        circ, net, path, prec = configs.serve_request_circuit(int(i))
        _, ops = path_cost(net, path.pairs, path.sliced)
        if ops <= 2 ** 28:                          # the oracle contracts a slice in well under a second
            sampled.append((int(i), circ, net, path, prec))
        if len(sampled) == 4:
            break
    assert len(sampled) == 4
    jobs = []       # (label, plan, tn, first, count, ref, tol, out)

    def add(label, net, path, prec, first, count, ref, tol):
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        plan = tnc.Plan(tn, path.pairs, path.sliced, tnc.PREC_BF16X3 if prec else tnc.PREC_C64)
        jobs.append((label, plan, tn, first, count, ref, tol, np.zeros(1, dtype=np.complex128)))

    # state vector: entry 41 (6 x 4 grid, depth 8, 4 slices, complex64)
    circ, net, path, prec = configs.serve_request_circuit(41)
    assert circ.n_qubits == 24 and prec == 0
    gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
    print("entry 41: state vector of 24 qubits", flush=True)
    sv = osv.amplitude(circ.n_qubits, gates, circ.bitstring)
    add("entry 41 vs state vector", net, path, 0, 0, int(np.prod([net.extents[l] for l in path.sliced])),
        [sv], 1e-5)
    # whole 25-qubit requests against the FP64 tensor-network oracle
    for i in (27, 29):
        circ, net, path, prec = configs.serve_request_circuit(i)
        assert circ.n_qubits == 25
        print(f"entry {i}: FP64 oracle over all slices", flush=True)
        ref = complex(oc.contract(net, path))
        tol = max(1e-5, 4 * 2.0 ** -16 * _tree_depth(net.n_leaves, path.pairs)) if prec else 1e-5
        add(f"entry {i} (prec {prec}) vs oracle", net, path, prec, 0,
            int(np.prod([net.extents[l] for l in path.sliced])), [ref], tol)
    # sampled slices of larger requests
    for i, circ, net, path, prec in sampled:
        n_sl = int(np.prod([net.extents[l] for l in path.sliced]))
        srng = np.random.Generator(np.random.PCG64(6000 + i))
        for s in (int(x) for x in srng.choice(n_sl, 3, replace=False)):
            print(f"entry {i} ({circ.n_qubits} qubits): oracle slice {s} of {n_sl}", flush=True)
            ref = complex(oc.contract(net, path, slices=[s]))
            tol = max(1e-5, 4 * 2.0 ** -16 * _tree_depth(net.n_leaves, path.pairs)) if prec else 1e-5
            add(f"entry {i} slice {s} (prec {prec})", net, path, prec, s, 1, [ref], tol)
    tnc.tnc_serve_start(ctx.handle, 8, 256)
    ids = [tnc.tnc_submit(ctx.handle, j[1].handle, j[3], j[4], j[7]) for j in jobs]
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    # per request: rms of its sampled references (one value for whole requests)
    groups = {}
    for j in jobs:
        groups.setdefault(j[0].split(" slice")[0], []).append(j)
    for key, js in groups.items():
        refs = np.array([j[5][0] for j in js])
        rms = float(np.sqrt(np.mean(np.abs(refs) ** 2)))
        for label, plan, tn, first, count, ref, tol, out in js:
            err = abs(complex(out[0]) - ref[0])
            print(f"{label}: |err| / rms {err / rms:.2e}, relative {err / abs(ref[0]):.2e} (tol {tol:.1e})",
                  flush=True)
            assert err <= tol * rms, label
    for j in jobs:
        j[1].close()
        j[2].close()
    ctx.close()


def test_served_graph_plans_match_eager(served):
    """Plans that replay their chunks as captured hipGraphs give, served
    concurrently, bitwise the eager result of the same plan alone."""
    ctx, pool, nets, plans = served
    order = list(range(len(plans)))
    alone = {}
    for i in order:
        o, _ = run_all(ctx, plans, [i], 1)
        alone[i] = o[i]
    gplans = []
    for i, (net, path) in enumerate(pool):
        p = tnc.Plan(nets[i], path.pairs, path.sliced)
        tnc.tnc_plan_set_graph(p.handle, True)
        gplans.append(p)
    rng = np.random.Generator(np.random.PCG64(8))
    mixed = [int(x) for x in rng.permutation(order)] * 2
    tnc.tnc_serve_start(ctx.handle, 6, 1024)
    outs, ids = [], []
    for i in mixed:
        out = np.zeros(1, dtype=np.complex128)
        outs.append((i, out))
        ids.append(tnc.tnc_submit(ctx.handle, gplans[i].handle, 0, gplans[i].info.n_slices, out))
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    for i, out in outs:
        assert np.array_equal(out.view(np.uint64), alone[i].view(np.uint64)), i
    for p in gplans:
        p.close()


def test_batcher_rows_match_batched_contract_and_state_vector():
    """Row requests of a batcher (circuit12 amplitude queries, B = 16 rows per
    batch), served among ordinary requests: each equals bitwise its row of a
    batched contraction of the same bitstrings on a separate network (so the
    row's batch position and its batch-mates do not matter), and the
    brute-force state vector within 1e-5.  Plans on the batcher's network
    are refused for ordinary submission."""
    from oracle import statevector as osv
    from workloads import configs
    from workloads.circuits import circuit_network_batched
    circ = configs.circuit12_circuit()
    nq, B, n_req = circ.n_qubits, 16, 40
    rng = np.random.Generator(np.random.PCG64(515))
    bits = rng.integers(0, 2, size=(n_req, nq))
    bits[24:28] = bits[0:4]                      # repeated queries
    arena = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    net = circuit_network_batched(circ, np.zeros((B, nq), dtype=np.int64))
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]   # projector of qubit q = carriers[q]
    path = greedy_path(net)
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    batcher = tnc.Batcher(plan, beta, carriers)

    # reference rows: batched contractions of the same bitstrings, B at a time
    tn_ref = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan_ref = tnc.Plan(tn_ref, path.pairs)
    ref = np.empty(n_req, dtype=np.complex128)
    for c0 in range(0, n_req, B):
        chunk = np.zeros((B, nq), dtype=np.int64)
        chunk[:min(B, n_req - c0)] = bits[c0:c0 + B]
        netc = circuit_network_batched(circ, chunk)
        for t in carriers:
            tn_ref.set_tensor(t, netc.leaves[t])
        ref[c0:c0 + B] = plan_ref.contract()[:min(B, n_req - c0)]

    others = [configs.circuit12()]
    other_plans = []
    for onet, opath in others:
        otn = tnc.Network(ctx, onet.labels, onet.extents, onet.open, onet.c64().leaves)
        other_plans.append((otn, tnc.Plan(otn, opath.pairs, opath.sliced)))
    other_alone = [p.contract().copy() for _, p in other_plans]

    tnc.tnc_serve_start(ctx.handle, 8, 1024)
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_submit(ctx.handle, plan.handle, 0, 1, np.zeros(B, dtype=np.complex128))
    assert e.value.status == tnc.E_BUSY
    outs, ids, oids = [], [], []
    eye = np.eye(2, dtype=np.complex128)
    for i in range(n_req):
        out = np.zeros(1, dtype=np.complex128)
        outs.append(out)
        ids.append(tnc.tnc_submit_row(ctx.handle, batcher.handle, [eye[bits[i, q]] for q in range(nq)], out))
        if i % 10 == 0:
            o = np.zeros(1, dtype=np.complex128)
            oids.append((tnc.tnc_submit(ctx.handle, other_plans[0][1].handle, 0, 1, o), o))
    lat = [tnc.tnc_wait(ctx.handle, rid) for rid in ids]
    for rid, _ in oids:
        tnc.tnc_wait(ctx.handle, rid)
    tnc.tnc_serve_stop(ctx.handle)
    print(f"batcher: {n_req} rows, p50 latency {1e3 * np.median(lat):.2f} ms", flush=True)

    got = np.array([o[0] for o in outs])
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert np.array_equal(got[24:28].view(np.uint64), got[0:4].view(np.uint64))
    for _, o in oids:
        assert np.array_equal(o.view(np.uint64), other_alone[0].view(np.uint64))
    gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
    sv = osv.run(nq, gates)
    for i in range(n_req):
        want = sv[tuple(int(x) for x in bits[i])]
        assert abs(got[i] - want) <= 1e-5 * abs(want), i
    batcher.close()
    for otn, p in other_plans:
        p.close()
        otn.close()
    plan_ref.close()
    plan.close()
    ctx.close()


def test_batcher_sliced_plan_odd_batch_and_early_destroy():
    """A batcher over a sliced plan (two sliced labels, every batch sums all
    slices in FP64) with B = 5 rows: 23 row requests match the state vector
    within 1e-5.  The batcher handle is destroyed while its rows are still
    queued (they run), and its network then takes ordinary requests again."""
    from oracle import statevector as osv
    from workloads import configs
    from workloads.circuits import circuit_network_batched
    circ = configs.circuit12_circuit()
    nq, B, n_req = circ.n_qubits, 5, 23
    bits = np.random.Generator(np.random.PCG64(77)).integers(0, 2, size=(n_req, nq))
    arena = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena.numel(), arena_ptr=arena.data_ptr())
    net = circuit_network_batched(circ, np.zeros((B, nq), dtype=np.int64))
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
    path = greedy_path(net)
    sl = greedy_slice(net, path.pairs, n_sliced=2)
    assert len(sl) == 2
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, sl)
    assert plan.info.n_slices == 4
    batcher = tnc.Batcher(plan, beta, carriers)
    eye = np.eye(2, dtype=np.complex128)
    tnc.tnc_serve_start(ctx.handle, 4, 256)
    outs = [np.zeros(1, dtype=np.complex128) for _ in range(n_req)]
    ids = [tnc.tnc_submit_row(ctx.handle, batcher.handle, [eye[bits[i, q]] for q in range(nq)], outs[i])
           for i in range(n_req)]
    batcher.close()                                   # rows still queued keep it alive
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    # the last row is done, so the network is free for ordinary requests again
    whole = np.zeros(B, dtype=np.complex128)
    tnc.tnc_wait(ctx.handle, tnc.tnc_submit(ctx.handle, plan.handle, 0, plan.info.n_slices, whole))
    tnc.tnc_serve_stop(ctx.handle)
    gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
    sv = osv.run(nq, gates)
    for i in range(n_req):
        want = sv[tuple(int(x) for x in bits[i])]
        assert abs(outs[i][0] - want) <= 1e-5 * abs(want), i
    plan.close()
    tn.close()
    ctx.close()


def test_poll_reports_completion_and_unknown_ids(served):
    """tnc_poll says "not done" (latency 0) until the request finishes, then
    done with its latency; the polled result equals the request alone; an id
    already collected by tnc_wait is unknown (TNC_E_ARG)."""
    import time
    ctx, pool, nets, plans = served
    alone, _ = run_all(ctx, plans, [1], 1)
    tnc.tnc_serve_start(ctx.handle, 2, 64)
    out = np.zeros(1, dtype=np.complex128)
    rid = tnc.tnc_submit(ctx.handle, plans[1].handle, 0, plans[1].info.n_slices, out)
    t0 = time.time()
    while True:
        done, lat = tnc.tnc_poll(ctx.handle, rid)
        if done:
            break
        assert lat == 0.0
        assert time.time() - t0 < 60, "request did not finish"
        time.sleep(0.0005)
    assert lat > 0.0
    assert tnc.tnc_wait(ctx.handle, rid) == lat
    with pytest.raises(tnc.TncError) as e:
        tnc.tnc_poll(ctx.handle, rid)
    assert e.value.status == tnc.E_ARG
    tnc.tnc_serve_stop(ctx.handle)
    assert np.array_equal(out.view(np.uint64), alone[1].view(np.uint64))


def test_concurrent_submitters_and_waiters(served):
    """The submit / submit_row / poll / wait calls are thread-safe: four
    Python threads (ctypes drops the GIL inside each call, so the calls
    overlap) submit ordinary requests and wait on or poll their own ids while
    a fifth submits batcher rows.  Every result equals bitwise the same
    request served alone, and every row its row of a batched contraction."""
    import threading

    from workloads import configs
    from workloads.circuits import circuit_network_batched
    ctx, pool, nets, plans = served
    alone = {}
    for i in range(len(plans)):
        o, _ = run_all(ctx, plans, [i], 1)
        alone[i] = o[i]

    circ = configs.circuit12_circuit()
    nq, B, n_rows = circ.n_qubits, 8, 24
    net = circuit_network_batched(circ, np.zeros((B, nq), dtype=np.int64))
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
    path = greedy_path(net)
    bits = np.random.Generator(np.random.PCG64(616)).integers(0, 2, size=(n_rows, nq))
    tn_ref = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan_ref = tnc.Plan(tn_ref, path.pairs)
    ref = np.empty(n_rows, dtype=np.complex128)
    for c0 in range(0, n_rows, B):
        netc = circuit_network_batched(circ, bits[c0:c0 + B])
        for t in carriers:
            tn_ref.set_tensor(t, netc.leaves[t])
        ref[c0:c0 + B] = plan_ref.contract()
    tn_b = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan_b = tnc.Plan(tn_b, path.pairs)
    batcher = tnc.Batcher(plan_b, beta, carriers)

    errors, results, rows_out = [], [], np.zeros(n_rows, dtype=np.complex128)
    lock = threading.Lock()
    eye = np.eye(2, dtype=np.complex128)

    def submitter(t):
        try:
            rng = np.random.Generator(np.random.PCG64(900 + t))
            mine = []
            for i in (int(x) for x in rng.integers(0, len(plans), size=8)):
                out = np.zeros(1, dtype=np.complex128)
                mine.append((i, out, tnc.tnc_submit(ctx.handle, plans[i].handle, 0, plans[i].info.n_slices, out)))
            for n, (i, out, rid) in enumerate(mine):
                if n % 2:
                    while not tnc.tnc_poll(ctx.handle, rid)[0]:
                        pass
                tnc.tnc_wait(ctx.handle, rid)
            with lock:
                results.extend((i, out) for i, out, _ in mine)
        except Exception as e:  # noqa: BLE001 - reported by the main thread
            errors.append(repr(e))

    def row_submitter():
        try:
            outs = [rows_out[i:i + 1] for i in range(n_rows)]
            rids = [tnc.tnc_submit_row(ctx.handle, batcher.handle, [eye[bits[i, q]] for q in range(nq)], outs[i])
                    for i in range(n_rows)]
            for rid in rids:
                tnc.tnc_wait(ctx.handle, rid)
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    tnc.tnc_serve_start(ctx.handle, 6, 1024)
    threads = [threading.Thread(target=submitter, args=(t,)) for t in range(4)]
    threads.append(threading.Thread(target=row_submitter))
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=90)
    alive = [th.is_alive() for th in threads]
    tnc.tnc_serve_stop(ctx.handle)
    assert not any(alive), alive
    assert not errors, errors
    assert len(results) == 32
    for i, out in results:
        assert np.array_equal(out.view(np.uint64), alone[i].view(np.uint64)), i
    assert np.array_equal(rows_out.view(np.uint64), ref.view(np.uint64))
    batcher.close()
    plan_b.close()
    tn_b.close()
    plan_ref.close()
    tn_ref.close()


def _serve_each(ctx, items, fuse, flops_per_launch=tnc.FUSE_ALL):
    """Serve (plan, first, count) items with one slot; with `fuse`, a slow
    request queued first lets the items queue up behind it, so that the
    worker admits them together (by default every light request of one
    structure is fused, launch-bound or not).  Returns the outputs and the
    server's (jobs, fused jobs, fused requests)."""
    tnc.tnc_serve_start(ctx.handle, 1, 1024)
    tnc.tnc_serve_set_fusion(ctx.handle, 8 if fuse else 1, flops_per_launch)
    blocker = None
    if fuse:
        circ = random_circuit(6, 6, 10, seed=8100)       # 1.5e12 FLOP: ~10 ms of work ahead of the items
        net = circuit_network(circ)
        path = greedy_path(net)
        sl = greedy_slice(net, path.pairs, n_sliced=4)
        btn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        bplan = tnc.Plan(btn, path.pairs, sl)
        bout = np.zeros(1, dtype=np.complex128)
        blocker = (btn, bplan, tnc.tnc_submit(ctx.handle, bplan.handle, 0, bplan.info.n_slices, bout))
    outs = [np.zeros(p.info.n_result, dtype=np.complex128) for p, _, _ in items]
    ids = [tnc.tnc_submit(ctx.handle, p.handle, f, c, o) for (p, f, c), o in zip(items, outs)]
    if blocker:
        tnc.tnc_wait(ctx.handle, blocker[2])
    for rid in ids:
        tnc.tnc_wait(ctx.handle, rid)
    stats = tnc.tnc_serve_get_stats(ctx.handle)
    tnc.tnc_serve_stop(ctx.handle)
    if blocker:
        blocker[1].close()
        blocker[0].close()
    return outs, stats


@pytest.mark.parametrize("prec, form", [(tnc.PREC_C64, tnc.GEMM_4M), (tnc.PREC_C64, tnc.GEMM_3M),
                                        (tnc.PREC_BF16X3, tnc.GEMM_4M), (tnc.PREC_BF16X3, tnc.GEMM_3M)],
                         ids=["4M", "3M", "bf16x3", "bf16x3_3M"])
def test_fused_requests_are_bitwise_alone(served, prec, form):
    """Light requests of one structure run as one fused job (each tree
    level's small GEMMs and gathers one launch over all of them, every MFMA
    step one grouped launch where its tile has a grouped form, else one
    launch per request): (i) six 5x5-grid circuits of depth 10
    with different gates and bitstrings (same network shape, so the same
    path, slicing and plan structure), four slices each; (ii) one sliced
    network's slices as four requests of one chunk each.  Every result is
    bitwise the one the request gets alone, and matches the oracle."""
    ctx = served[0]
    nets, items, refs, handles = [], [], [], []
    for seed in range(6):
        circ = random_circuit(5, 5, 10, seed=8200 + seed)
        net = circuit_network(circ)
        path = greedy_path(net)
        sl = greedy_slice(net, path.pairs, n_sliced=2)
        nets.append((net, Path(path.pairs, sl)))
    # one structure: every network has the same path and slicing
    assert all(np.array_equal(n[1].pairs, nets[0][1].pairs) and n[1].sliced == nets[0][1].sliced for n in nets)
    for net, path in nets:
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        p = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
        handles.append((tn, p))
        items.append((p, 0, p.info.n_slices))
        refs.append(complex(oc.contract(net, path)))
    # one network's four slices, one chunk (one slice) per request
    net, path = nets[0]
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    ps = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
    tnc.tnc_plan_set_max_chunk(ps.handle, 1)
    ps.info = tnc.tnc_plan_get_info(ps.handle)
    handles.append((tn, ps))
    for s in range(ps.info.n_slices):
        items.append((ps, s, 1))
        refs.append(complex(oc.contract(net, path, slices=[s])))
    n_mfma = sum(tnc.tnc_plan_get_batch_step(items[0][0].handle, s).kernel == 0
                 for s in range(items[0][0].info.n_steps))
    assert n_mfma >= 3
    print(f"fusion: {len(items)} requests, {n_mfma} MFMA steps per chunk", flush=True)
    alone, st_alone = _serve_each(ctx, items, fuse=False)
    mix, st_mix = _serve_each(ctx, items, fuse=True)
    print(f"fusion: alone {st_alone}, mixed {st_mix}", flush=True)
    assert st_alone[1] == 0
    assert st_mix[1] >= 2 and st_mix[2] >= 6
    for i, (a, m) in enumerate(zip(alone, mix)):
        assert np.array_equal(a.view(np.uint64), m.view(np.uint64)), i
    depth = _tree_depth(nets[0][0].n_leaves, nets[0][1].pairs)
    tol = 1e-5 if prec == tnc.PREC_C64 else max(1e-5, (8 if form == tnc.GEMM_3M else 4) * 2.0 ** -16 * depth)
    rms = np.sqrt(np.mean(np.abs(np.array(refs[6:])) ** 2))
    for i, (m, ref) in enumerate(zip(mix, refs)):
        scale = abs(ref) if i < 6 else rms     # single slices: Porter-Thomas, bounded by the rms
        assert abs(complex(m[0]) - ref) <= tol * scale, (i, complex(m[0]), ref)
    for tn, p in handles:
        p.close()
        tn.close()


@pytest.mark.parametrize("prec, form", [(tnc.PREC_C64, tnc.GEMM_4M), (tnc.PREC_BF16X3, tnc.GEMM_4M),
                                        (tnc.PREC_BF16X3, tnc.GEMM_3M)], ids=["4M", "bf16x3", "bf16x3_3M"])
def test_fused_jobs_through_every_grouped_tile_variant(served, prec, form):
    """Every tile variant forced on every MFMA step (tnc_ctx_set_gemm_variant)
    while six 4x5-grid circuits of depth 10 run as one fused job: the steps
    whose variant has a grouped form (every 4M variant; split precision's
    0, 4, 5, 6 in the 4M form, all but 3 in the 3M form) run as grouped
    launches, the others one launch per request.  Every result is bitwise
    the one the request gets alone with the same variant."""
    ctx = served[0]
    items, handles = [], []
    for seed in range(6):
        net = circuit_network(random_circuit(4, 5, 10, seed=8400 + seed))
        path = greedy_path(net)
        sl = greedy_slice(net, path.pairs, n_sliced=1)
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        p = tnc.Plan(tn, path.pairs, sl, prec, form)
        handles.append((tn, p))
        items.append((p, 0, p.info.n_slices))
    assert any(tnc.tnc_plan_get_batch_step(items[0][0].handle, s).kernel == 0
               for s in range(items[0][0].info.n_steps))
    try:
        for variant in range(7):
            tnc.tnc_ctx_set_gemm_variant(ctx.handle, variant)
            alone, _ = _serve_each(ctx, items, fuse=False)
            mix, st = _serve_each(ctx, items, fuse=True)
            print(f"variant {variant}: fused {st}", flush=True)
            assert st[1] >= 1 and st[2] >= 2
            for i, (a, m) in enumerate(zip(alone, mix)):
                assert np.array_equal(a.view(np.uint64), m.view(np.uint64)), (variant, i)
    finally:
        tnc.tnc_ctx_set_gemm_variant(ctx.handle, -1)
    for tn, p in handles:
        p.close()
        tn.close()


def test_fusion_takes_only_launch_bound_requests(served):
    """The server's default criterion fuses a light request only below 2^30
    planned FLOP per launch of its own run: six 4x5-grid circuits of depth
    10 (2.4e8 FLOP over 18 launches) queued behind a slow request run as one
    fused job; six 5x6-grid circuits of depth 10 (9.8e10 FLOP over 24
    launches, light but bound by arithmetic) queued with them run one by
    one.  Every result is bitwise the one the request gets alone."""
    ctx = served[0]
    items, handles, launch_bound = [], [], []
    for rows, cols in ((4, 5), (5, 6)):
        ns = 1 if rows == 4 else 2
        for seed in range(6):
            net = circuit_network(random_circuit(rows, cols, 10, seed=8300 + seed))
            path = greedy_path(net)
            sl = greedy_slice(net, path.pairs, n_sliced=ns)
            tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
            p = tnc.Plan(tn, path.pairs, sl)
            handles.append((tn, p))
            items.append((p, 0, p.info.n_slices))
            info = tnc.tnc_plan_get_info(p.handle)
            launch_bound.append(info.flops_per_slice * info.n_slices < info.n_launches * tnc.FUSE_FLOPS_PER_LAUNCH)
    assert launch_bound == [True] * 6 + [False] * 6
    alone, _ = _serve_each(ctx, items, fuse=False)
    mix, st = _serve_each(ctx, items, fuse=True, flops_per_launch=tnc.FUSE_FLOPS_PER_LAUNCH)
    print(f"fusion criterion: {st}", flush=True)
    assert st == (1 + 1 + 6, 1, 6)       # blocker, one fused job of the six 4x5 circuits, six 5x6 alone
    for i, (a, m) in enumerate(zip(alone, mix)):
        assert np.array_equal(a.view(np.uint64), m.view(np.uint64)), i
    for tn, p in handles:
        p.close()
        tn.close()
