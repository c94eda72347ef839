"""Benchmark: complex TFLOP/s of path execution on one MI355X.

Workload (default): single large pairwise contractions, complex64, all mode
extents 2, i.i.d. complex Gaussian entries --
  * A with 30 modes x B with 28 modes, 14 shared (output 2^30 entries), both
    stored in seeded random mode orders so that the operand permutations
    precede the GEMM (m = 2^16, n = 2^14, k = 2^14);
  * a batch of 64 contractions with 20 / 18 modes, 10 shared
    (h = 64, m = 2^10, n = 2^8, k = 2^10).
One step = one execution of both paths (all operand permutations, the
batched complex GEMMs on MFMA, results written to HBM).  Inputs are resident
in HBM before timing starts.  FLOPs follow the paper's convention of 8 real
FLOPs per complex multiply-add.

Prints one JSON line.  ``roofline`` is for the dominant kernel (the large
GEMM), its launch time measured with HIP events on its own stream over the
timed steps; ``cpu_baseline`` times the FP64 oracle on a bounded sample of
the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM_TBS = 8.0       # TB/s, MI355X HBM3E
PEAK_BF16_MFMA = 2516.6  # TFLOP/s, MI355X dense bf16 matrix
PEAK_HBM = 8000.0        # GB/s

# Memory-side traffic per launch of the dominant kernel (4M GEMM, 4x4-wave
# tiles, the 2^30-output contraction), from rocprofv3 --pmc FETCH_SIZE
# (333,213,036 KiB, x2.0) and WRITE_SIZE (8,388,610 KiB, x1.0); the factors
# are what the same counters read for a 4 GiB device copy.  FETCH_SIZE counts
# every L2 miss (served by the MALL or HBM): with k = 2^14 the A/B panels of
# the tiles running at once are re-read per K stage.  Set to None when the
# kernel changes.
GEMM_TRAFFIC_BYTES = 691.0e9


def path_roofline_s(tnc, plan, n_runs: int = 1, leaf_permutes: bool = True) -> float:
    """The Sec. IV cost model as the path's roofline: every step of one
    device batch at max(its algorithmic bytes 8 (hA m k + hB n k + h m n) /
    8 TB/s, its FLOPs 8 h m n k / 157.3 TFLOP/s), plus the leaf permutes at
    16 bytes per element / 8 TB/s; times the number of batches run."""
    info = tnc.tnc_plan_get_info(plan.handle)
    t = 0.0
    for s in range(info.n_steps):
        st = tnc.tnc_plan_get_batch_step(plan.handle, s)
        fl = 8.0 * st.h * st.m * st.n * st.k
        by = 8.0 * (st.hA * st.m * st.k + st.hB * st.n * st.k + st.h * st.m * st.n)
        t += max(by / (PEAK_HBM_TBS * 1e12), fl / (PEAK_FP32_MFMA * 1e12))
    if leaf_permutes:
        t += info.transpose_bytes / (PEAK_HBM_TBS * 1e12)
    return t * n_runs


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", choices=["4M", "3M"], default="4M")
    ap.add_argument("--prec", choices=["c64", "bf16x3"], default="c64")
    ap.add_argument("--scale", type=int, default=0, help="drop this many modes from each group (smaller run)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["pair30", "circuit40", "serve", "small"], default="pair30")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-latency leg")
    ap.add_argument("--no-forms", action="store_true", help="skip timing the 3M and split-bf16 forms")
    ap.add_argument("--amp-queries", action="store_true",
                    help="with --workload small: also serve 4096 amplitude queries through batchers "
                         "(off by default: one run under rocprofv3 --kernel-trace ended in a host SIGSEGV "
                         "whose cause is not found)")
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--slices", type=int, default=0, help="circuit40: slices per run (0 = all)")
    ap.add_argument("--arena-gib", type=float, default=64.0, help="circuit40: arena size")
    ap.add_argument("--max-chunk", type=int, default=0, help="circuit40: cap on slices per batch")
    ap.add_argument("--graph", action="store_true", help="circuit40: replay chunks as hipGraphs")
    ap.add_argument("--probe-copy", action="store_true",
                    help="after timing, run one 4 GiB device-to-device copy (calibrates HBM counters)")
    return ap.parse_args()


def cpu_baseline(net_a, path_a, net_b, path_b, n_fixed: int = 4):
    """The oracle (complex128 numpy) on a bounded sample: the big contraction
    with its n_fixed leading M labels fixed to one value (1/16 of the rows
    for 4, 10-25 s on 16 host threads) and 4 of the 64 batch entries.
    Rate = sample FLOPs (8 per complex MAC) / time."""
    from oracle import contract as oc
    from workloads.network import Network, Path

    t_total, flops_total = 0.0, 0.0
    # big pair: fix the leading M labels (open labels; taken as a sub-network)
    a, b = net_a.leaves
    la, lb = net_a.labels
    fix = {l: 0 for l in range(n_fixed)}
    idx = tuple(0 if l in fix else slice(None) for l in la)
    sub_a = np.ascontiguousarray(a[idx])
    sub_la = tuple(l for l in la if l not in fix)
    sub = Network([sub_a, b], [sub_la, lb], net_a.extents, tuple(l for l in net_a.open if l not in fix))
    t0 = time.perf_counter()
    oc.contract(sub, Path(path_a.pairs, ()))
    dt = time.perf_counter() - t0
    m_sub = int(np.prod([net_a.extents[l] for l in sub_la])) // (2 ** 14)
    t_total += dt
    flops_total += 8.0 * m_sub * 2 ** 14 * 2 ** 14
    # batch pair: 4 of the 64 entries
    a2, b2 = net_b.leaves
    sub2 = Network([a2[:4], b2[:4]], net_b.labels, net_b.extents.copy(), net_b.open)
    sub2.extents[net_b.open[0]] = 4
    t0 = time.perf_counter()
    oc.contract(sub2, path_b)
    dt2 = time.perf_counter() - t0
    t_total += dt2
    flops_total += 8.0 * 4 * 1024 * 256 * 1024
    threads, host = host_description()
    return {"value": flops_total / t_total / 1e12, "unit": "complex TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"pair30 rows with {n_fixed} leading M labels fixed (1/{2 ** n_fixed} of the work, {dt:.1f} s) + 4 of 64 "
                      f"batch entries ({dt2:.1f} s); numpy complex128 tensordot incl. operand transposes; {host}"}


def host_description():
    """(BLAS threads, "CPU model, BLAS library") of this process."""
    from threadpoolctl import threadpool_info
    pools = threadpool_info()
    threads = max((i.get("num_threads", 1) for i in pools), default=1)
    blas = ", ".join(sorted({f"{i.get('internal_api', '?')} {i.get('version') or ''}".strip() for i in pools})) or "?"
    cpu = "?"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "?")
    except OSError:
        pass
    return int(threads), f"{cpu}, BLAS {blas}"


def cpu_baseline_slices(net, path, flops_per_slice: float, n_slices: int, n_sample: int = 128):
    """The oracle on a bounded sample of the sliced workload: n_sample seeded
    random slices, each contracted alone along the path (numpy complex128,
    as the paper's per-slice loop would), about 10 s on 16 host threads.
    Rate = the sample's FLOPs (the plan's per-slice count, 8 per complex
    MAC) / time."""
    from oracle import contract as oc
    rng = np.random.Generator(np.random.PCG64(1040))
    sample = [int(x) for x in rng.choice(n_slices, min(n_sample, n_slices), replace=False)]
    t0 = time.perf_counter()
    for s in sample:
        oc.contract(net, path, slices=[s])
    dt = time.perf_counter() - t0
    threads, host = host_description()
    return {"value": flops_per_slice * len(sample) / dt / 1e12, "unit": "complex TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(sample)} of {n_slices} slices, each alone ({dt:.1f} s, {dt / len(sample) * 1e3:.0f} ms "
                      f"per slice: {dt / len(sample) * n_slices:.0f} s extrapolated to all); numpy complex128 "
                      f"tensordot; {host}"}


HEAVY_FLOPS = 2.0 ** 38   # requests planned at >= this many FLOP share one heavy slot


def serving_leg(args):
    """Serving mix: a pool of random grid circuits (20..48 qubits, depth 8..14,
    4^j slices, complex64 or split-bf16, planned work capped at 2^43 FLOP),
    Poisson arrivals at ``load`` x the measured saturation throughput of the
    continuous-batching server (heavy requests, >= 2^38 planned FLOP, in a
    lane of one slot); the same arrival trace is replayed through the server
    without the heavy lane and with one slot (one request at a time), at the
    main load and at 0.5 and 0.95 of saturation.  Latency is submit to
    done, measured by the library."""
    import threading

    import torch

    from paper_2606_01852_amd import tnc
    from workloads import configs

    log(f"serving: building a pool of {args.serve_pool} circuits")
    t0 = time.time()
    pool = [configs.serve_request(i) for i in range(args.serve_pool)]
    log(f"serving: pool ready in {time.time() - t0:.1f} s")
    arena_bytes = 64 << 30
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena_bytes, arena_ptr=arena.data_ptr())
    nets, plans, flops = [], [], []
    for net, path, prec in pool:
        tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
        p = tnc.Plan(tn, path.pairs, path.sliced, tnc.PREC_BF16X3 if prec else tnc.PREC_C64, tnc.GEMM_4M)
        tnc.tnc_plan_set_max_chunk(p.handle, 256)
        tnc.tnc_plan_autotune(p.handle)
        p.info = tnc.tnc_plan_get_info(p.handle)
        nets.append(tn)
        plans.append(p)
        flops.append(p.info.chunk_flops * (p.info.n_slices // p.info.max_chunk))
    rng = np.random.Generator(np.random.PCG64(99))
    which = [int(x) for x in rng.integers(0, len(plans), args.serve_requests)]
    gaps = rng.exponential(1.0, args.serve_requests)
    outs = [np.zeros(1, dtype=np.complex128) for _ in which]

    def replay(slots, arrivals, heavy=HEAVY_FLOPS):
        tnc.tnc_serve_start(ctx.handle, slots, 1 << 16)
        tnc.tnc_serve_set_heavy(ctx.handle, heavy, 1)
        t_start = time.perf_counter()
        ids = []
        for i, (w, at) in enumerate(zip(which, arrivals)):
            delay = t_start + at - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids.append(tnc.tnc_submit(ctx.handle, plans[w].handle, 0, plans[w].info.n_slices, outs[i]))
        lat = [tnc.tnc_wait(ctx.handle, r) for r in ids]
        t_end = time.perf_counter()
        tnc.tnc_serve_stop(ctx.handle)
        return np.array(lat), t_end - t_start

    # warm up every plan once (tables, kernels)
    replay(args.serve_slots, np.zeros(len(which)))
    lat_sat, t_sat = replay(args.serve_slots, np.zeros(len(which)))
    sat = len(which) / t_sat
    servers = (("continuous_batching", args.serve_slots, HEAVY_FLOPS),
               ("continuous_no_heavy_lane", args.serve_slots, 0.0),
               ("one_at_a_time", 1, 0.0))
    tot_flops = sum(flops[w] for w in which)

    def measure(load):
        rate = load * sat
        arrivals = np.cumsum(gaps) / rate
        log(f"serving: saturation {sat:.1f} req/s; replaying {len(which)} Poisson arrivals at {rate:.1f} req/s")
        out = {}
        for name, slots, heavy in servers:
            lat, wall = replay(slots, arrivals, heavy)
            out[name] = {"slots": slots, "heavy_lane_flops": heavy,
                         "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                         "req_per_s": round(len(which) / wall, 2),
                         "tflops": round(tot_flops / wall / 1e12, 3)}
            log(f"serving {name} at load {load}: {out[name]}")
        return out, rate

    res, rate = measure(args.serve_load)
    res["other_loads"] = {}
    for load in (0.5, 0.95):
        if load != args.serve_load:
            r, _ = measure(load)
            res["other_loads"][str(load)] = {k: {"p50_ms": v["p50_ms"], "p99_ms": v["p99_ms"]} for k, v in r.items()}
    res["arrival_rate_req_per_s"] = round(rate, 2)
    res["saturation_req_per_s"] = round(sat, 2)
    res["requests"] = len(which)
    res["pool"] = len(plans)
    for p in plans:
        p.close()
    for n in nets:
        n.close()
    ctx.close()
    del arena
    torch.cuda.empty_cache()
    return res


def bench_small(args):
    """Latency-bound and mixed workloads: the 12-qubit circuit amplitude
    (153 tiny steps, 13 tree levels) step by step or level-grouped, eager or
    replayed as a hipGraph; 64 bitstrings as one batched network; all 4096
    amplitudes with the
    FP64 norm, and the closed 8x8 bond-4 grid in complex64, 3M and split-bf16."""
    import torch

    from paper_2606_01852_amd import tnc
    from workloads import configs
    from workloads.circuits import circuit_network
    from workloads.grids import prescale_log2
    from workloads.network import Network
    from workloads.paths import greedy_path

    ctx = tnc.Context(0, arena_bytes=8 << 30, stream=torch.cuda.current_stream().cuda_stream)
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    net, path = configs.circuit12()
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    for grouping in (False, True):
        for graph in (False, True):
            p = tnc.Plan(tn, path.pairs)
            tnc.tnc_plan_set_grouping(p.handle, grouping)
            tnc.tnc_plan_set_graph(p.handle, graph)
            dt = timed(lambda: p.contract(), 200)
            key = f"circuit12_amplitude_{'grouped' if grouping else 'stepwise'}_{'graph' if graph else 'eager'}_us"
            out[key] = round(dt * 1e6, 1)
            p.close()
    circ = configs.circuit12_circuit()
    from workloads.circuits import circuit_network_batched
    bits = np.random.Generator(np.random.PCG64(64)).integers(0, 2, size=(64, circ.n_qubits))
    netb = circuit_network_batched(circ, bits)
    tnb = tnc.Network(ctx, netb.labels, netb.extents, netb.open, netb.c64().leaves)
    pb = tnc.Plan(tnb, greedy_path(netb).pairs)
    tnc.tnc_plan_set_graph(pb.handle, True)
    dt = timed(lambda: pb.contract(), 100)
    out["circuit12_64_bitstrings_one_plan_us"] = round(dt * 1e6, 1)
    pb.close()
    netall = circuit_network(circ, open_qubits=range(12))
    pathall = greedy_path(netall)
    tna = tnc.Network(ctx, netall.labels, netall.extents, netall.open, netall.c64().leaves)
    pa = tnc.Plan(tna, pathall.pairs)
    tnc.tnc_plan_set_graph(pa.handle, True)
    dt = timed(lambda: pa.contract(), 100)
    out["circuit12_all_4096_amplitudes_us"] = round(dt * 1e6, 1)
    out["circuit12_norm2_minus_1"] = tnc.tnc_plan_result_norm2(pa.handle) - 1.0

    g, _ = configs.grid8()
    e = prescale_log2(g.labels)
    gs = Network([x * 2.0 ** int(k) for x, k in zip(g.leaves, e)], g.labels, g.extents, ())
    gpath = greedy_path(gs)
    tg = tnc.Network(ctx, gs.labels, gs.extents, gs.open, gs.c64().leaves)
    for name, prec, form in (("c64_4M", tnc.PREC_C64, tnc.GEMM_4M), ("c64_3M", tnc.PREC_C64, tnc.GEMM_3M),
                             ("bf16x3", tnc.PREC_BF16X3, tnc.GEMM_4M)):
        p = tnc.Plan(tg, gpath.pairs, (), prec, form)
        tnc.tnc_plan_autotune(p.handle)
        tnc.tnc_plan_set_graph(p.handle, True)
        dt = timed(lambda: p.contract(), 20)
        out[f"grid8_{name}_ms"] = round(dt * 1e3, 3)
        out[f"grid8_{name}_tflops"] = round(p.info.flops_per_slice / dt / 1e12, 3)
        p.close()
    if args.amp_queries:
        out["amplitude_queries"] = amplitude_query_leg(ctx)
    print(json.dumps({"small_workloads": out}), flush=True)


def amplitude_query_leg(ctx, n_queries: int = 4096):
    """circuit12 amplitude queries (random bitstrings) served as row requests
    through the library's server (8 slots): one batcher of 64 rows per batch
    (dynamic batching: the queued queries' same-shape steps share each
    launch) vs 8 batchers of one row (one query per run, up to 8 running at
    once).  A burst of all queries gives the saturation rate (submission from
    this Python thread included); Poisson streams at 0.5 and 3 x the one-row
    servers' saturation give p50/p99 latency (submit to done, measured by the
    library).  Rows are checked against 64-row batched contractions."""
    import ctypes as C

    from paper_2606_01852_amd import tnc
    from workloads import configs
    from workloads.circuits import circuit_network_batched
    from workloads.paths import greedy_path

    circ = configs.circuit12_circuit()
    nq = circ.n_qubits
    rng = np.random.Generator(np.random.PCG64(4096))
    bits = rng.integers(0, 2, size=(n_queries, nq))
    eye = [np.ascontiguousarray(np.eye(2, dtype=np.complex128)[b]) for b in (0, 1)]
    ptr_rows = [(C.c_void_p * nq)(*[eye[int(x)].ctypes.data for x in bits[i]]) for i in range(n_queries)]
    outs = np.zeros(n_queries, dtype=np.complex128)
    out_ptrs = [outs[i:].ctypes.data_as(C.POINTER(C.c_double)) for i in range(n_queries)]
    L = tnc.lib()

    def make(B, copies):
        made = []
        for _ in range(copies):
            net = circuit_network_batched(circ, np.zeros((B, nq), dtype=np.int64))
            beta = net.open[0]
            carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
            tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
            p = tnc.Plan(tn, greedy_path(net).pairs)
            tnc.tnc_plan_set_graph(p.handle, True)
            made.append((tn, p, tnc.Batcher(p, beta, carriers)))
        return made

    def replay(made, arrivals):
        tnc.tnc_serve_start(ctx.handle, 8, 1 << 16)
        rid = C.c_uint64()
        ids = []
        t_start = time.perf_counter()
        for i, at in enumerate(arrivals):
            delay = t_start + at - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            b = made[i % len(made)][2].handle
            st = L.tnc_submit_row(ctx.handle, b, ptr_rows[i], tnc.IN_C128, out_ptrs[i], C.byref(rid))
            if st != tnc.OK:
                raise tnc.TncError(st, L.tnc_last_error().decode())
            ids.append(rid.value)
        lat = np.array([tnc.tnc_wait(ctx.handle, r) for r in ids])
        wall = time.perf_counter() - t_start
        tnc.tnc_serve_stop(ctx.handle)
        return lat, wall

    servers = {"batched_64_rows": make(64, 1), "one_row_x8": make(1, 8)}
    res, sat, got = {}, {}, {}
    for name, made in servers.items():
        replay(made, np.zeros(256))                      # warm-up: tables, graphs
        lat, wall = replay(made, np.zeros(n_queries))
        sat[name] = n_queries / wall
        got[name] = outs.copy()
        res[name] = {"burst_queries_per_s": round(sat[name], 1)}
        log(f"amplitude queries {name}: burst of {n_queries} at {sat[name]:.0f} queries/s")
    # the bursts' rows against 64-row batched contractions of the same bitstrings
    ref = np.empty(n_queries, dtype=np.complex128)
    net = circuit_network_batched(circ, bits[:64])
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    p = tnc.Plan(tn, greedy_path(net).pairs)
    for c0 in range(0, n_queries, 64):
        netc = circuit_network_batched(circ, bits[c0:c0 + 64])
        for t in carriers:
            tn.set_tensor(t, netc.leaves[t])
        ref[c0:c0 + 64] = p.contract()
    res["batched_rows_bitwise_equal_to_contraction"] = bool(
        np.array_equal(got["batched_64_rows"].view(np.uint64), ref.view(np.uint64)))
    res["one_row_rel_frobenius_diff"] = float(np.linalg.norm(got["one_row_x8"] - ref) / np.linalg.norm(ref))
    p.close()
    tn.close()
    gaps = rng.exponential(1.0, n_queries)
    for load in (0.5, 3.0):
        rate = load * sat["one_row_x8"]
        arrivals = np.cumsum(gaps) / rate
        for name, made in servers.items():
            lat, wall = replay(made, arrivals)
            res[name][f"rate_{load}x"] = {"queries_per_s": round(rate, 1),
                                          "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 1),
                                          "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 1)}
            log(f"amplitude queries {name} at {rate:.0f}/s: {res[name][f'rate_{load}x']}")
    for made in servers.values():
        for tn, p, b in made:
            b.close()
            p.close()
            tn.close()
    return res


def bench_circuit40(args):
    """Sliced 40-qubit circuit (5x8 grid, depth 12, 16 sliced labels = 65,536
    slices): the slices run as a batch dimension of every step, summed in FP64."""
    import torch

    from paper_2606_01852_amd import tnc
    from workloads import configs

    log("building circuit40 network, path and slices")
    net, path = configs.circuit40()
    stream = torch.cuda.current_stream()
    arena_bytes = int(args.arena_gib * (1 << 30))
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    ctx = tnc.Context(0, arena_bytes=arena_bytes, arena_ptr=arena.data_ptr(), stream=stream.cuda_stream)
    prec = tnc.PREC_BF16X3 if args.prec == "bf16x3" else tnc.PREC_C64
    form = tnc.GEMM_3M if args.form == "3M" else tnc.GEMM_4M
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
    if args.max_chunk:
        tnc.tnc_plan_set_max_chunk(plan.handle, args.max_chunk)
    if args.graph:
        tnc.tnc_plan_set_graph(plan.handle, True)
    t_tune = time.time()
    tnc.tnc_plan_autotune(plan.handle)
    log(f"autotuned in {time.time() - t_tune:.1f} s")
    info = tnc.tnc_plan_get_info(plan.handle)
    n = args.slices or info.n_slices
    log(f"slices {n} of {info.n_slices}; chunk {info.max_chunk}; chunk peak {info.chunk_peak_bytes / 2**30:.1f} GiB; "
        f"{info.flops_per_slice:.3e} FLOP per slice")
    for _ in range(args.warmup):
        plan.contract(0, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z = plan.contract(0, n)
    dt = (time.perf_counter() - t0) / args.steps
    tnc.tnc_plan_set_profile(plan.handle, True)
    plan.contract(0, n)
    per_step = []
    for s in range(info.n_steps):
        ms, cnt = tnc.tnc_plan_get_profile(plan.handle, s)
        per_step.append((ms, s))
    perm_ms, perm_n = tnc.tnc_plan_get_profile(plan.handle, -1)
    red_ms, red_n = tnc.tnc_plan_get_profile(plan.handle, -2)
    per_step.sort(reverse=True)
    tot = sum(x[0] for x in per_step)
    log(f"profiled run: GEMMs {tot:.1f} ms, leaf permutes {perm_ms:.1f} ms ({perm_n}), reductions {red_ms:.2f} ms")
    n_chunks = max(1, n // info.max_chunk)
    for ms, s in per_step[:12]:
        st = tnc.tnc_plan_get_batch_step(plan.handle, s)
        f = 8.0 * st.h * st.m * st.n * st.k * n_chunks
        log(f"  step {s:4d}: {ms:8.2f} ms  h {st.h} m {st.m} n {st.n} k {st.k} kernel {st.kernel} "
            f"variant {st.variant} split {st.split} swapped {st.swapped}: {f / ms / 1e9:.1f} TFLOP/s")
    exec_flops = info.chunk_flops * n_chunks if n % info.max_chunk == 0 else info.flops_per_slice * n
    value = exec_flops / dt / 1e12
    log(f"executed {exec_flops:.3e} FLOP ({info.flops_per_slice * n:.3e} without hoisting slice-invariant steps)")
    # outputs written in their consumer's order by the GEMM epilogue: an
    # executor storing [H|M|N] would transpose them (read + write) instead
    perm_steps, avoided = 0, 0.0
    for s in range(info.n_steps):
        st = tnc.tnc_plan_get_batch_step(plan.handle, s)
        if not st.natural:
            perm_steps += 1
            avoided += 16.0 * st.h * st.m * st.n * n_chunks
    log(f"{perm_steps} of {info.n_steps} steps store in consumer order: {avoided / 1e9:.1f} GB of transposes avoided")
    roof_s = path_roofline_s(tnc, plan, n_chunks, leaf_permutes=False)
    log(f"path roofline (GEMM steps of the batched run): {roof_s * 1e3:.1f} ms = {roof_s / dt:.3f} of the measured")
    # the same slices contracted one at a time (a chunk of one slice), the
    # per-slice loop whose cost the paper projects as t_slice * 2^b
    single = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
    tnc.tnc_plan_set_max_chunk(single.handle, 1)
    tnc.tnc_plan_set_graph(single.handle, True)
    tnc.tnc_plan_autotune(single.handle)
    n_loop = 32
    for i in range(2):
        single.contract(i, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(n_loop):
        single.contract(i, 1)
    torch.cuda.synchronize()
    t_slice = (time.perf_counter() - t1) / n_loop
    single.close()
    log(f"one slice at a time: {t_slice * 1e3:.2f} ms per slice -> {t_slice * n:.1f} s for {n} slices "
        f"(batched: {dt:.2f} s, {t_slice * n / dt:.1f}x)")
    res = {"metric": "complex TFLOP/s of path execution (% MFMA peak) + p50/p99 request latency",
           "value": round(value, 3), "unit": "complex TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64/fp32" if prec == tnc.PREC_C64 else "c64/bf16x3",
           "data": "synthetic",
           "config": {"workload": "circuit40: 5x8 grid, depth 12, 16 sliced labels", "slices": n,
                      "chunk": info.max_chunk, "amplitude": [z[0].real, z[0].imag],
                      "permuted_store_steps": perm_steps, "transposes_avoided_gb": round(avoided / 1e9, 2),
                      "per_slice_equivalent_tflops": round(info.flops_per_slice * n / dt / 1e12, 3),
                      "path_roofline_frac": round(roof_s / dt, 4),
                      "slice_loop_ms_per_slice": round(t_slice * 1e3, 3),
                      "slice_loop_extrapolated_s": round(t_slice * n, 2),
                      "batched_speedup_vs_slice_loop": round(t_slice * n / dt, 2)}}
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample of slices)")
        res["cpu_baseline"] = cpu_baseline_slices(net, path, info.flops_per_slice, info.n_slices)
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this executor runs on one GPU; multi-GPU execution is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "circuit40":
        return bench_circuit40(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "serve":
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return
    import torch

    from paper_2606_01852_amd import tnc
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    log("generating inputs")
    t0 = time.time()
    net_a, path_a = configs.pair30(scale=args.scale)
    net_b, path_b = configs.pair_batch(64, scale=args.scale)
    log(f"inputs ready in {time.time() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    prec = tnc.PREC_BF16X3 if args.prec == "bf16x3" else tnc.PREC_C64
    form = tnc.GEMM_3M if args.form == "3M" else tnc.GEMM_4M

    # plan on the host first to size the arena
    hctx = tnc.Context(-1)
    sizes = []
    for net, path in ((net_a, path_a), (net_b, path_b)):
        tn = tnc.Network(hctx, net.labels, net.extents, net.open)
        p = tnc.Plan(tn, path.pairs, (), prec, form)
        sizes.append(p.info.peak_bytes)
        p.close()
        tn.close()
    arena_bytes = max(sizes) + (64 << 20)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    ctx = tnc.Context(0, arena_bytes=arena_bytes, arena_ptr=arena.data_ptr(), stream=stream.cuda_stream)
    hw = tnc.tnc_device_calibrate(ctx.handle)
    log(f"measured ceilings: FP32 MFMA {hw.flops_per_s / 1e12:.1f} TFLOP/s, copy {hw.hbm_bytes_per_s / 1e9:.0f} GB/s")
    log("uploading leaves")
    tn_a = tnc.Network(ctx, net_a.labels, net_a.extents, net_a.open, net_a.leaves)
    tn_b = tnc.Network(ctx, net_b.labels, net_b.extents, net_b.open, net_b.leaves)
    plan_a = tnc.Plan(tn_a, path_a.pairs, (), prec, form)
    plan_b = tnc.Plan(tn_b, path_b.pairs, (), prec, form)
    log("autotuning tile shapes")
    t_tune = time.time()
    tnc.tnc_plan_autotune(plan_a.handle)
    tnc.tnc_plan_autotune(plan_b.handle)
    log(f"autotuned in {time.time() - t_tune:.1f} s: big GEMM variant {tnc.tnc_plan_get_step(plan_a.handle, 0).variant}, "
        f"batch GEMM variant {tnc.tnc_plan_get_step(plan_b.handle, 0).variant}")
    out_a = torch.empty(plan_a.info.n_result, dtype=torch.complex64, device=dev)
    out_b = torch.empty(plan_b.info.n_result, dtype=torch.complex64, device=dev)
    flops_step = plan_a.info.flops_per_slice + plan_b.info.flops_per_slice

    def step():
        tnc.tnc_contract_async(plan_a.handle, 0, 1, out_a.data_ptr(), tnc.OUT_C64)
        tnc.tnc_contract_async(plan_b.handle, 0, 1, out_b.data_ptr(), tnc.OUT_C64)

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tnc.tnc_plan_set_profile(plan_a.handle, True)
    tnc.tnc_plan_set_profile(plan_b.handle, True)
    log("timing")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gemm_ms, gemm_n = tnc.tnc_plan_get_profile(plan_a.handle, 0)
    perm_ms, perm_n = tnc.tnc_plan_get_profile(plan_a.handle, -1)
    bgemm_ms, bgemm_n = tnc.tnc_plan_get_profile(plan_b.handle, 0)
    bperm_ms, bperm_n = tnc.tnc_plan_get_profile(plan_b.handle, -1)
    gemm_avg_s = gemm_ms / max(gemm_n, 1) / 1e3
    achieved = plan_a.info.flops_per_slice / gemm_avg_s / 1e12
    peak = PEAK_BF16_MFMA / 3 if prec == tnc.PREC_BF16X3 else PEAK_FP32_MFMA
    value = flops_step * args.steps / dt / 1e12
    perm_bytes = plan_a.info.transpose_bytes
    perm_gbs = perm_bytes / (perm_ms / max(perm_n, 1) * 2 / 1e3) / 1e9 if perm_n else None
    log(f"step {dt / args.steps * 1e3:.1f} ms; big GEMM {gemm_avg_s * 1e3:.1f} ms = {achieved:.1f} TF; "
        f"permutes {perm_ms / max(perm_n, 1):.2f} ms/launch ({perm_gbs} GB/s avg over A,B); "
        f"batch GEMM {bgemm_ms / max(bgemm_n, 1):.3f} ms, batch permutes {bperm_ms / max(bperm_n, 1):.3f} ms")
    res = {
        "metric": "complex TFLOP/s of path execution (% MFMA peak) + p50/p99 request latency",
        "value": round(value, 3),
        "unit": "complex TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64/fp32" if prec == tnc.PREC_C64 else "c64/bf16x3",
        "data": "synthetic",
        "config": {"workload": "pair30+pair_batch64: A 30 modes x B 28 modes (14 shared, 2^30 outputs) and "
                               "64 x (20 x 18 modes, 10 shared); extents 2; random stored mode orders",
                   "form": args.form, "prec": args.prec, "scale": args.scale,
                   "pct_fp32_mfma_peak": round(100 * value / PEAK_FP32_MFMA, 1),
                   "path_roofline_frac": round((path_roofline_s(tnc, plan_a) + path_roofline_s(tnc, plan_b))
                                               / (dt / args.steps), 4)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(peak, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": GEMM_TRAFFIC_BYTES},
        "measured_ceilings": {"fp32_mfma_tflops": round(hw.flops_per_s / 1e12, 2),
                              "copy_gbs": round(hw.hbm_bytes_per_s / 1e9, 1),
                              "gemm_frac_of_measured_mfma": round(achieved / (hw.flops_per_s / 1e12), 4),
                              "permute_frac_of_measured_copy": round(perm_gbs / (hw.hbm_bytes_per_s / 1e9), 4)
                              if perm_gbs else None},
        "kernels": {"gemm_ms": round(gemm_avg_s * 1e3, 3),
                    "permute_ms_per_launch": round(perm_ms / max(perm_n, 1), 3),
                    "batch_gemm_ms": round(bgemm_ms / max(bgemm_n, 1), 3)},
    }
    if not args.no_forms and args.form == "4M" and args.prec == "c64":
        # the same step in the other GEMM forms (same inputs, same arena)
        res["other_forms"] = {}
        for name, fprec, fform, fpeak in (("3M", tnc.PREC_C64, tnc.GEMM_3M, PEAK_FP32_MFMA),
                                          ("bf16x3", tnc.PREC_BF16X3, tnc.GEMM_4M, PEAK_BF16_MFMA / 3)):
            pa = tnc.Plan(tn_a, path_a.pairs, (), fprec, fform)
            pb = tnc.Plan(tn_b, path_b.pairs, (), fprec, fform)
            tnc.tnc_plan_autotune(pa.handle)
            tnc.tnc_plan_autotune(pb.handle)

            def fstep():
                tnc.tnc_contract_async(pa.handle, 0, 1, out_a.data_ptr(), tnc.OUT_C64)
                tnc.tnc_contract_async(pb.handle, 0, 1, out_b.data_ptr(), tnc.OUT_C64)

            fstep()
            torch.cuda.synchronize()
            tnc.tnc_plan_set_profile(pa.handle, True)
            t1 = time.perf_counter()
            for _ in range(2):
                fstep()
            torch.cuda.synchronize()
            fdt = (time.perf_counter() - t1) / 2
            g_ms, g_n = tnc.tnc_plan_get_profile(pa.handle, 0)
            g_s = g_ms / max(g_n, 1) / 1e3
            res["other_forms"][name] = {
                "tflops": round(flops_step / fdt / 1e12, 3), "ms_per_step": round(fdt * 1e3, 3),
                "gemm_tflops": round(plan_a.info.flops_per_slice / g_s / 1e12, 3),
                "gemm_frac_of_form_peak": round(plan_a.info.flops_per_slice / g_s / 1e12 / fpeak, 4),
                "variant": tnc.tnc_plan_get_step(pa.handle, 0).variant}
            log(f"form {name}: {res['other_forms'][name]}")
            pa.close()
            pb.close()
    if args.probe_copy:
        src = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 4 GiB read + 4 GiB written")
        del src, dst
    if not args.no_serve:
        plan_a.close()
        plan_b.close()
        tn_a.close()
        tn_b.close()
        ctx.close()
        del arena
        torch.cuda.empty_cache()
        res["latency"] = serving_leg(args)
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample)")
        res["cpu_baseline"] = cpu_baseline(net_a, path_a, net_b, path_b)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
