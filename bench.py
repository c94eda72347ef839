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
the same workload on this host's cores, and ``error_vs_oracle`` compares the
GPU's rows of that sample with the oracle's.  ``configs`` holds one record
for each other workload (the 12-qubit circuit amplitude, the 8x8 bond-4
grid, the sliced 40-qubit circuit), each with its measured error against the
FP64 oracle, its roofline and its own CPU-oracle baseline; ``latency`` is the
serving mix (continuous batching vs one request at a time).
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
# (371,296,253 KiB, x2.0) and WRITE_SIZE (8,388,609 KiB, x1.0); the factors
# are what the same counters read for a 4 GiB device copy.  FETCH_SIZE counts
# every L2 miss (served by the memory-side cache or HBM): with k = 2^14 the
# A/B panels of the tiles running at once are re-read per K stage.  Set to
# None when the kernel changes.
GEMM_TRAFFIC_BYTES = 769.0e9


def path_roofline_s(tnc, plan, n_runs: int = 1, leaf_permutes: bool = True, split: bool = False,
                    three_m: bool = False) -> float:
    """The Sec. IV cost model as the path's roofline: every step of one
    device batch at max(its algorithmic bytes 8 (hA m k + hB n k + h m n) /
    8 TB/s, its MFMA work / the precision's peak), plus the leaf permutes at
    16 bytes per element / 8 TB/s; times the number of batches run.  MFMA
    work: 8 h m n k FLOP (6 h m n k executed in the 3M form) at 157.3
    TFLOP/s, or at 2516.6 / 3 for split precision (three bf16 products per
    real product)."""
    info = tnc.tnc_plan_get_info(plan.handle)
    peak = (PEAK_BF16_MFMA / 3 if split else PEAK_FP32_MFMA) * 1e12
    t = 0.0
    for s in range(info.n_steps):
        st = tnc.tnc_plan_get_batch_step(plan.handle, s)
        fl = (6.0 if three_m else 8.0) * st.h * st.m * st.n * st.k
        by = 8.0 * (st.hA * st.m * st.k + st.hB * st.n * st.k + st.h * st.m * st.n)
        t += max(by / (PEAK_HBM_TBS * 1e12), fl / peak)
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
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-arena-gib", type=float, default=240.0,
                    help="serving: arena size (the admission budget for planned intermediates)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-workload records (circuit12, grid8, circuit40)")
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--slices", type=int, default=0, help="circuit40: slices per run (0 = all)")
    ap.add_argument("--arena-gib", type=float, default=160.0, help="circuit40: arena size")
    ap.add_argument("--max-chunk", type=int, default=0, help="circuit40: cap on slices per batch")
    ap.add_argument("--graph", action="store_true", help="circuit40: replay chunks as hipGraphs")
    ap.add_argument("--counters", action="store_true",
                    help="circuit40: only the timed runs (default tile variants, no profiled run, no comparisons, "
                         "no error checks): for rocprofv3 counter passes")
    ap.add_argument("--store-order", type=int, choices=[0, 1], default=0,
                    help="circuit40: 1 = store interleaved outputs through a separate transpose instead of the "
                         "GEMM's permuted-store epilogue (to measure what the epilogue saves)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="after timing, run one 4 GiB device-to-device copy (calibrates HBM counters)")
    return ap.parse_args()


def cpu_baseline(net_a, path_a, net_b, path_b, n_fixed: int = 4):
    """The oracle (complex128 numpy) on a bounded sample: the big contraction
    with its n_fixed leading M labels fixed to 0 (the first 1/16 of the
    result rows for 4, 10-25 s on 16 host threads) and 4 of the 64 batch
    entries.  Rate = sample FLOPs (8 per complex MAC) / time.  Returns the
    record and the oracle's results (those rows, those batch entries)."""
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
    ref_rows = oc.contract(sub, Path(path_a.pairs, ()))
    dt = time.perf_counter() - t0
    m_sub = int(np.prod([net_a.extents[l] for l in sub_la])) // (2 ** 14)
    t_total += dt
    flops_total += 8.0 * m_sub * 2 ** 14 * 2 ** 14
    # batch pair: 4 of the 64 entries
    a2, b2 = net_b.leaves
    sub2 = Network([a2[:4], b2[:4]], net_b.labels, net_b.extents.copy(), net_b.open)
    sub2.extents[net_b.open[0]] = 4
    t0 = time.perf_counter()
    ref_batch = oc.contract(sub2, path_b)
    dt2 = time.perf_counter() - t0
    t_total += dt2
    flops_total += 8.0 * 4 * 1024 * 256 * 1024
    threads, host = host_description()
    rec = {"value": flops_total / t_total / 1e12, "unit": "complex TFLOP/s", "cores": threads,
           "kind": "oracle",
           "sample": f"pair30 rows with {n_fixed} leading M labels fixed (1/{2 ** n_fixed} of the work, {dt:.1f} s) + 4 of 64 "
                     f"batch entries ({dt2:.1f} s); numpy complex128 tensordot incl. operand transposes; {host}"}
    return rec, np.asarray(ref_rows).reshape(-1), np.asarray(ref_batch).reshape(-1)


def rel_err(got, ref):
    """(relative Frobenius error, max elementwise error / max |ref|)."""
    got = np.asarray(got, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    d = np.abs(got - ref)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), float(d.max() / np.abs(ref).max())


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
    refs = np.empty(len(sample), dtype=np.complex128)
    t0 = time.perf_counter()
    for i, s in enumerate(sample):
        refs[i] = complex(oc.contract(net, path, slices=[s]))
    dt = time.perf_counter() - t0
    threads, host = host_description()
    rec = {"value": flops_per_slice * len(sample) / dt / 1e12, "unit": "complex TFLOP/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{len(sample)} of {n_slices} slices, each alone ({dt:.1f} s, {dt / len(sample) * 1e3:.0f} ms "
                     f"per slice: {dt / len(sample) * n_slices:.0f} s extrapolated to all); numpy complex128 "
                     f"tensordot; {host}"}
    return rec, sample, refs


HEAVY_FLOPS = 2.0 ** 38   # requests planned at >= this many FLOP share one heavy slot


def _pool_entry(i: int):
    from workloads import configs
    return configs.serve_request(i)


def build_pool(n: int):
    """The serving pool's networks and paths (greedy path and slicer per
    circuit), built in 16 worker processes: the path search dominates and
    runs on the host only."""
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=min(16, n), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_pool_entry, range(n)))


def serving_leg(args):
    """Serving mix (config 4): a pool of random grid circuits (20..48 qubits,
    depth 8..14, 4^j slices, complex64 or split-bf16, planned work capped at
    2^43 FLOP), admitted by planned arena bytes within a 240 GiB arena.
    Closed-loop saturation (all requests queued at once) of the
    continuous-batching server (8 slots, heavy requests of >= 2^38 planned
    FLOP in a lane of one slot) and of the one-request-at-a-time server; then
    the same seeded Poisson arrival trace (2,000 requests drawn from the
    pool) replayed at 0.5, 0.8 and 0.95 x the continuous server's
    saturation through both, and at 0.8 through the continuous server without
    the heavy lane.  Latency is submit to done, measured by the library."""
    import torch

    from paper_2606_01852_amd import tnc

    log(f"serving: building a pool of {args.serve_pool} circuits (16 processes)")
    t0 = time.time()
    pool = build_pool(args.serve_pool)
    log(f"serving: pool ready in {time.time() - t0:.1f} s")
    arena_bytes = int(args.serve_arena_gib * (1 << 30))
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
    tot_flops = sum(flops[w] for w in which)

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

    def stats(lat, wall):
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "req_per_s": round(len(lat) / wall, 2), "tflops": round(tot_flops / wall / 1e12, 3)}

    # warm up every plan once (tables, kernels, graphs)
    replay(args.serve_slots, np.zeros(len(which)))
    burst = np.zeros(len(which))
    sat = {}
    for name, slots, heavy in (("continuous_batching", args.serve_slots, HEAVY_FLOPS), ("one_at_a_time", 1, 0.0)):
        lat, wall = replay(slots, burst, heavy)
        sat[name] = stats(lat, wall)
        log(f"serving: closed-loop saturation of {name}: {sat[name]}")
    rate0 = sat["continuous_batching"]["req_per_s"]
    res = {"saturation": sat}
    for load in (0.5, 0.8, 0.95):
        rate = load * rate0
        arrivals = np.cumsum(gaps) / rate
        servers = [("continuous_batching", args.serve_slots, HEAVY_FLOPS), ("one_at_a_time", 1, 0.0)]
        if load == 0.8:
            servers.insert(1, ("continuous_no_heavy_lane", args.serve_slots, 0.0))
        res[f"load_{load}"] = {"arrival_rate_req_per_s": round(rate, 2)}
        for name, slots, heavy in servers:
            lat, wall = replay(slots, arrivals, heavy)
            res[f"load_{load}"][name] = stats(lat, wall)
            log(f"serving {name} at load {load} ({rate:.1f} req/s): {res[f'load_{load}'][name]}")
    res["requests"] = len(which)
    res["pool"] = len(plans)
    res["arena_gib"] = args.serve_arena_gib
    res["fusion"] = fusion_leg(ctx, tnc)
    res["slots"] = args.serve_slots
    res["heavy_lane_flops"] = HEAVY_FLOPS
    for p in plans:
        p.close()
    for n in nets:
        n.close()
    ctx.close()
    del arena
    torch.cuda.empty_cache()
    return res


def fusion_leg(ctx, tnc, n: int = 512):
    """Light requests of one structure, queued all at once through the
    8-slot server, with fusion of up to 8 same-structure requests per job
    and without; the results are compared bitwise.  Three mixes of 64 random
    circuits each (different gates and bitstrings, one network shape, so one
    path and slicing), by planned FLOP per launch of a request's own run:
    4x5-grid circuits of depth 10 (1 sliced label, 2.4e8 FLOP over 18
    launches per amplitude: launch-bound), 5x5 of depth 10 (2 sliced labels,
    8.9e9 over 20) and 5x6 of depth 10 (2 sliced labels, 9.8e10 over 24:
    bound by the GPU's arithmetic).  Where the server's default criterion
    does not fuse a mix, forced fusion is timed for comparison."""
    from workloads.circuits import circuit_network, random_circuit
    from workloads.paths import greedy_path, greedy_slice

    res = {"requests": n, "circuits": 64, "slots": 8, "max_fused": 8,
           "flops_per_launch_criterion": tnc.FUSE_FLOPS_PER_LAUNCH}
    for name, rows, cols, n_sl in (("launch_bound_4x5_d10", 4, 5, 1), ("mixed_5x5_d10", 5, 5, 2),
                                   ("gpu_bound_5x6_d10", 5, 6, 2)):
        circs = [random_circuit(rows, cols, 10, seed=9000 + i) for i in range(64)]
        nets = [circuit_network(c) for c in circs]
        path = greedy_path(nets[0])               # structure only: the same for every circuit
        sl = greedy_slice(nets[0], path.pairs, n_sliced=n_sl)
        tns = [tnc.Network(ctx, x.labels, x.extents, x.open, x.c64().leaves) for x in nets]
        plans = [tnc.Plan(t, path.pairs, sl) for t in tns]
        for p in plans:
            p.info = tnc.tnc_plan_get_info(p.handle)
        flops = plans[0].info.flops_per_slice * plans[0].info.n_slices
        r = {"flops_per_request": flops, "launches_per_request": plans[0].info.n_launches}
        outs = {}
        legs = [("warmup", 8, tnc.FUSE_ALL), ("unfused", 1, tnc.FUSE_ALL), ("fused_8", 8, tnc.FUSE_FLOPS_PER_LAUNCH)]
        if flops >= plans[0].info.n_launches * tnc.FUSE_FLOPS_PER_LAUNCH:
            legs.append(("fused_8_forced", 8, tnc.FUSE_ALL))
        for leg, fuse, per_launch in legs:
            tnc.tnc_serve_start(ctx.handle, 8, 1 << 16)
            tnc.tnc_serve_set_fusion(ctx.handle, fuse, per_launch)
            o = [np.zeros(1, dtype=np.complex128) for _ in range(n)]
            t0 = time.perf_counter()
            ids = [tnc.tnc_submit(ctx.handle, plans[i % 64].handle, 0, plans[i % 64].info.n_slices, o[i])
                   for i in range(n)]
            lat = np.array([tnc.tnc_wait(ctx.handle, q) for q in ids])
            wall = time.perf_counter() - t0
            jobs, fj, fr = tnc.tnc_serve_get_stats(ctx.handle)
            tnc.tnc_serve_stop(ctx.handle)
            outs[leg] = np.array([x[0] for x in o])
            r[leg] = {"req_per_s": round(n / wall, 1), "tflops": round(n * flops / wall / 1e12, 3),
                      "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                      "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                      "jobs": jobs, "fused_jobs": fj, "fused_requests": fr}
            log(f"fusion leg {name} {leg}: {r[leg]}")
        del r["warmup"]
        r["bitwise_equal"] = all(bool(np.array_equal(outs[k].view(np.uint64), outs["unfused"].view(np.uint64)))
                                 for k in outs if k != "unfused")
        r["fused_over_unfused"] = round(r["fused_8"]["req_per_s"] / r["unfused"]["req_per_s"], 3)
        res[name] = r
        for p in plans:
            p.close()
        for t in tns:
            t.close()
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
                             ("bf16x3", tnc.PREC_BF16X3, tnc.GEMM_4M), ("bf16x3_3M", tnc.PREC_BF16X3, tnc.GEMM_3M)):
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


def dominant_step(tnc, plan, split: bool = False, three_m: bool = False):
    """The step with the most profiled kernel time (profiling on, a run just
    done): its algorithmic bytes 8 (hA m k + hB n k + h m n) and FLOPs
    8 h m n k per batch, what bounds it at MI355X peaks (HBM 8 TB/s; MFMA:
    FP32 157.3 TFLOP/s, or bf16 2516.6 / 3 for split precision, three bf16
    products per real product) and the achieved fraction of that bound; for
    the 3M form also the fraction in executed MFMA work (6 of the 8 FLOPs
    per complex MAC)."""
    info = tnc.tnc_plan_get_info(plan.handle)
    best = None
    for s in range(info.n_steps):
        ms, cnt = tnc.tnc_plan_get_profile(plan.handle, s)
        if cnt and (best is None or ms > best[0]):
            best = (ms, cnt, s)
    if best is None:
        return None
    ms, cnt, s = best
    st = tnc.tnc_plan_get_batch_step(plan.handle, s)
    per = ms / cnt * 1e-3
    fl = 8.0 * st.h * st.m * st.n * st.k
    by = 8.0 * (st.hA * st.m * st.k + st.hB * st.n * st.k + st.h * st.m * st.n)
    peak_mfma = PEAK_BF16_MFMA / 3 if split else PEAK_FP32_MFMA
    mfma = fl / (peak_mfma * 1e12) >= by / (PEAK_HBM_TBS * 1e12)
    achieved = fl / per / 1e12 if mfma else by / per / 1e9
    peak = peak_mfma if mfma else PEAK_HBM
    rec = {"step": s, "h": st.h, "m": st.m, "n": st.n, "k": st.k, "kernel": st.kernel, "variant": st.variant,
           "ms_per_launch": round(per * 1e3, 4), "launches": cnt, "bound": "mfma" if mfma else "hbm",
           "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": "TFLOP/s" if mfma else "GB/s",
           "frac": round(achieved / peak, 4)}
    if mfma and three_m:
        rec["frac_executed"] = round(achieved * 6 / 8 / peak, 4)
    return rec


def oracle_time(fn, reps: int = 3) -> float:
    """Median wall time of the oracle call (seconds)."""
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def record_circuit12():
    """Config 0: the 12-qubit 3x4 circuit of depth 8 as a closed amplitude
    network (154 leaves, greedy path), complex64 4M, level-grouped and
    replayed as a hipGraph: latency of one amplitude and of all 4096 (open
    network, FP64 norm on the device), each with its error against the FP64
    oracle; the amplitude also against the state vector, and unitarity.
    Latency-bound: the roofline is the path's Eq. (6) time at peak rates
    (nanoseconds) against the measured latency."""
    import torch

    from oracle import contract as oc
    from oracle import statevector as osv
    from paper_2606_01852_amd import tnc
    from workloads import configs
    from workloads.circuits import circuit_network
    from workloads.paths import greedy_path

    ctx = tnc.Context(0, arena_bytes=1 << 30, stream=torch.cuda.current_stream().cuda_stream)
    circ = configs.circuit12_circuit()
    net, path = configs.circuit12()
    tn = tnc.Network(ctx, net.labels, net.extents, net.open, net.c64().leaves)
    plan = tnc.Plan(tn, path.pairs)
    tnc.tnc_plan_set_graph(plan.handle, True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    dt = timed(lambda: plan.contract(), 500)
    amp = complex(plan.contract()[0])
    ref = complex(oc.contract(net, path))
    gates = [(qs, u.astype(np.complex64).astype(np.complex128)) for qs, u in circ.gates]
    sv = osv.amplitude(circ.n_qubits, gates, circ.bitstring)
    roof = path_roofline_s(tnc, plan)
    netall = circuit_network(circ, open_qubits=range(12))
    pathall = greedy_path(netall)
    tna = tnc.Network(ctx, netall.labels, netall.extents, netall.open, netall.c64().leaves)
    pa = tnc.Plan(tna, pathall.pairs)
    tnc.tnc_plan_set_graph(pa.handle, True)
    dt_all = timed(lambda: pa.contract(), 200)
    amps = pa.contract()
    norm2 = tnc.tnc_plan_result_norm2(pa.handle)
    ref_all = oc.contract(netall, pathall).reshape(-1)
    e_all, e_all_max = rel_err(amps, ref_all)
    t_cpu = oracle_time(lambda: oc.contract(net, path), 5)
    threads, host = host_description()
    rec = {"workload": "circuit12: 3x4 grid, depth 8, closed amplitude network, greedy path (153 steps)",
           "latency_us": round(dt * 1e6, 2), "unit": "us per amplitude", "dtype": "c64/fp32",
           "tflops": round(plan.info.flops_per_slice / dt / 1e12, 6),
           "error_vs_oracle": abs(amp - ref) / abs(ref), "error_vs_statevector": abs(amp - sv) / abs(sv),
           "tolerance": 1e-5,
           "all_4096_amplitudes": {"latency_us": round(dt_all * 1e6, 2), "rel_frobenius_error_vs_oracle": e_all,
                                   "max_error_over_max_amplitude": e_all_max,
                                   "sum_abs2_minus_1": norm2 - 1.0},
           "roofline": {"bound": "latency", "path_roofline_us": round(roof * 1e6, 4),
                        "measured_us": round(dt * 1e6, 2), "frac": round(roof / dt, 6)},
           "cpu_baseline": {"value": round(t_cpu * 1e6, 1), "unit": "us per amplitude", "cores": threads,
                            "kind": "oracle", "sample": f"the same amplitude, median of 5; {host}"}}
    for h in (plan, tn, pa, tna, ctx):
        h.close()
    return rec


def record_grid8():
    """Config 2: the closed 8x8 grid network of bond dimension 4 (64 leaves,
    greedy path) contracted to a scalar in complex64 4M, 3M and
    split-bf16x3 (exact power-of-two leaf prescaling, undone in FP64); each
    with its error against the FP64 oracle (and split-bf16x3 against the
    oracle's split emulation), the path roofline, the dominant step's
    roofline, and the oracle's time for the same contraction."""
    import torch

    from oracle import contract as oc
    from oracle import split as osp
    from paper_2606_01852_amd import tnc
    from workloads import configs
    from workloads.grids import prescale_log2
    from workloads.network import Network
    from workloads.paths import greedy_path

    ctx = tnc.Context(0, arena_bytes=8 << 30, stream=torch.cuda.current_stream().cuda_stream)
    g, _ = configs.grid8()
    e = prescale_log2(g.labels)
    gs = Network([x * 2.0 ** int(k) for x, k in zip(g.leaves, e)], g.labels, g.extents, ())
    gpath = greedy_path(gs)
    depth = [0] * gs.n_leaves
    for a, b in gpath.pairs:
        depth.append(1 + max(depth[int(a)], depth[int(b)]))
    exact = complex(oc.contract(gs, gpath))
    emu = complex(oc.contract(gs, gpath, step=osp.split_step))
    t_cpu = oracle_time(lambda: oc.contract(gs, gpath), 3)
    tg = tnc.Network(ctx, gs.labels, gs.extents, gs.open, gs.c64().leaves)
    threads, host = host_description()
    rec = {"workload": "grid8: closed 8x8 grid, bond 4, CN(0,1)/sqrt(numel) entries (x 2^floor(deg/2), exact), "
                       "greedy path (63 steps)", "forms": {}}
    for name, prec, form in (("c64_4M", tnc.PREC_C64, tnc.GEMM_4M), ("c64_3M", tnc.PREC_C64, tnc.GEMM_3M),
                             ("bf16x3", tnc.PREC_BF16X3, tnc.GEMM_4M), ("bf16x3_3M", tnc.PREC_BF16X3, tnc.GEMM_3M)):
        p = tnc.Plan(tg, gpath.pairs, (), prec, form)
        tnc.tnc_plan_autotune(p.handle)
        tnc.tnc_plan_set_graph(p.handle, True)
        p.contract()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            z = complex(p.contract()[0])
        dt = (time.perf_counter() - t0) / 20
        p2 = tnc.Plan(tg, gpath.pairs, (), prec, form)
        tnc.tnc_plan_autotune(p2.handle)
        tnc.tnc_plan_set_profile(p2.handle, True)
        p2.contract()
        dom = dominant_step(tnc, p2, prec == tnc.PREC_BF16X3, form == tnc.GEMM_3M)
        roof = path_roofline_s(tnc, p, split=prec == tnc.PREC_BF16X3, three_m=form == tnc.GEMM_3M)
        flops = p.info.flops_per_slice
        f = {"ms": round(dt * 1e3, 4), "tflops": round(flops / dt / 1e12, 3),
             "error_vs_oracle": abs(z - exact) / abs(exact), "path_roofline_frac": round(roof / dt, 4),
             "dominant_step": dom}
        if prec == tnc.PREC_BF16X3:
            e = emu
            if form == tnc.GEMM_3M:   # MFMA steps in the 3M split form, small (VALU) steps in the 4M one
                kinds = iter([tnc.tnc_plan_get_step(p.handle, s).kernel for s in range(len(gpath.pairs))])
                e = complex(oc.contract(gs, gpath, step=lambda *a: (osp.split_step_3m if next(kinds) == 0
                                                                     else osp.split_step)(*a)))
            f["error_vs_split_emulation"] = abs(z - e) / abs(e)
            f["tolerance"] = max(1e-5, (8 if form == tnc.GEMM_3M else 4) * 2.0 ** -16 * depth[-1])
        else:
            f["tolerance"] = 1e-5
        rec["forms"][name] = f
        log(f"grid8 {name}: {f}")
        p.close()
        p2.close()
    rec["cpu_baseline"] = {"value": round(flops / t_cpu / 1e12, 6),
                           "unit": "complex TFLOP/s", "cores": threads, "kind": "oracle",
                           "sample": f"the whole contraction ({t_cpu * 1e3:.1f} ms, median of 3); {host}"}
    tg.close()
    ctx.close()
    return rec


def circuit40_record(args, steps: int, warmup: int, with_cpu: bool):
    """Config 3: the sliced 40-qubit circuit (5x8 grid, depth 12, 16 sliced
    labels = 65,536 slices) with the slices as a batch dimension of every
    step, summed in FP64; throughput, path and dominant-step rooflines, the
    per-slice loop it replaces, and errors against the FP64 oracle on
    sampled slices and on the sum of slices [0, 64)."""
    import torch

    from oracle import contract as oc
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
    if args.store_order:
        tnc.tnc_plan_set_store_order(plan.handle, args.store_order)
    t_tune = time.time()
    if not args.counters:
        tnc.tnc_plan_autotune(plan.handle)
    log(f"autotuned in {time.time() - t_tune:.1f} s")
    info = tnc.tnc_plan_get_info(plan.handle)
    n = args.slices or info.n_slices
    log(f"slices {n} of {info.n_slices}; chunk {info.max_chunk}; chunk peak {info.chunk_peak_bytes / 2**30:.1f} GiB; "
        f"{info.flops_per_slice:.3e} FLOP per slice")
    for _ in range(warmup):
        plan.contract(0, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        z = plan.contract(0, n)
    dt = (time.perf_counter() - t0) / steps
    if args.counters:
        log(f"counter run: {steps} runs of {n} slices at {dt * 1e3:.1f} ms, store order {args.store_order}")
        res = {"workload": "circuit40 counter run", "slices": n, "chunk": info.max_chunk,
               "store_order": args.store_order, "ms_per_run": round(dt * 1e3, 3), "amplitude": [z[0].real, z[0].imag]}
        plan.close()
        tn.close()
        ctx.close()
        del arena
        torch.cuda.empty_cache()
        return res
    n_chunks = max(1, n // info.max_chunk)
    prof = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
    if args.max_chunk:
        tnc.tnc_plan_set_max_chunk(prof.handle, args.max_chunk)
    tnc.tnc_plan_autotune(prof.handle)
    tnc.tnc_plan_set_profile(prof.handle, True)
    prof.contract(0, n)
    per_step = []
    for s in range(info.n_steps):
        ms, cnt = tnc.tnc_plan_get_profile(prof.handle, s)
        per_step.append((ms, s))
    perm_ms, perm_n = tnc.tnc_plan_get_profile(prof.handle, -1)
    red_ms, red_n = tnc.tnc_plan_get_profile(prof.handle, -2)
    per_step.sort(reverse=True)
    tot = sum(x[0] for x in per_step)
    log(f"profiled run: GEMMs {tot:.1f} ms, leaf permutes {perm_ms:.1f} ms ({perm_n}), reductions {red_ms:.2f} ms")
    for ms, s in per_step[:8]:
        st = tnc.tnc_plan_get_batch_step(plan.handle, s)
        f = 8.0 * st.h * st.m * st.n * st.k * n_chunks
        log(f"  step {s:4d}: {ms:8.2f} ms  h {st.h} m {st.m} n {st.n} k {st.k} kernel {st.kernel} "
            f"variant {st.variant} split {st.split} swapped {st.swapped}: {f / ms / 1e9:.1f} TFLOP/s")
    dom = dominant_step(tnc, prof, prec == tnc.PREC_BF16X3, form == tnc.GEMM_3M)
    prof.close()
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
    roof_s = path_roofline_s(tnc, plan, n_chunks, leaf_permutes=False, split=prec == tnc.PREC_BF16X3,
                             three_m=form == tnc.GEMM_3M)
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
    log(f"one slice at a time: {t_slice * 1e3:.2f} ms per slice -> {t_slice * n:.1f} s for {n} slices "
        f"(batched: {dt:.2f} s, {t_slice * n / dt:.1f}x)")
    res = {"workload": "circuit40: 5x8 grid, depth 12, 16 sliced labels", "slices": n,
           "value": round(value, 3), "unit": "complex TFLOP/s", "ms_per_run": round(dt * 1e3, 3),
           "steps": steps, "warmup": warmup,
           "dtype": "c64/fp32" if prec == tnc.PREC_C64 else "c64/bf16x3",
           "chunk": info.max_chunk, "amplitude": [z[0].real, z[0].imag],
           "permuted_store_steps": perm_steps, "transposes_avoided_gb": round(avoided / 1e9, 2),
           "per_slice_equivalent_tflops": round(info.flops_per_slice * n / dt / 1e12, 3),
           "path_roofline_frac": round(roof_s / dt, 4), "dominant_step": dom,
           "slice_loop_ms_per_slice": round(t_slice * 1e3, 3),
           "slice_loop_extrapolated_s": round(t_slice * n, 2),
           "batched_speedup_vs_slice_loop": round(t_slice * n / dt, 2)}
    # the executor without the permuted-store epilogue: interleaved outputs
    # stored in launch order and transposed by a separate launch (its
    # scratch buffers may shrink the chunk; both orders are timed at the
    # same chunk size)
    if args.store_order == 0:
        def timed_plan(order, cap):
            q = tnc.Plan(tn, path.pairs, path.sliced, prec, form)
            if cap:
                tnc.tnc_plan_set_max_chunk(q.handle, cap)
            tnc.tnc_plan_set_store_order(q.handle, order)
            tnc.tnc_plan_autotune(q.handle)
            zq = q.contract(0, n)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(steps):
                zq = q.contract(0, n)
            dq = (time.perf_counter() - t2) / steps
            cq = tnc.tnc_plan_get_info(q.handle).max_chunk
            q.close()
            return dq, zq, cq
        dt_alt, za, chunk_alt = timed_plan(1, args.max_chunk)
        if chunk_alt != info.max_chunk:
            dt_same, zs, _ = timed_plan(0, chunk_alt)
        else:
            dt_same, zs = dt, z
        res["separate_transpose_store"] = {
            "chunk": chunk_alt, "ms_per_run": round(dt_alt * 1e3, 3),
            "epilogue_ms_per_run_same_chunk": round(dt_same * 1e3, 3),
            "epilogue_saves_ms": round((dt_alt - dt_same) * 1e3, 3),
            "bitwise_equal": bool(np.array_equal(np.asarray(za).view(np.uint64), np.asarray(zs).view(np.uint64)))}
        log(f"separate-transpose store: {res['separate_transpose_store']}")
    # errors against the FP64 oracle: the sum of slices [0, 64) (FP64
    # accumulation on the device) and, with the CPU baseline, its sampled
    # slices one by one
    ref64 = sum(complex(oc.contract(net, path, slices=[s])) for s in range(64))
    got64 = complex(single.contract(0, 64)[0])
    res["error_vs_oracle"] = {"slices_0_64_sum_rel": abs(got64 - ref64) / abs(ref64)}
    if with_cpu:
        log("cpu baseline (oracle on a bounded sample of slices)")
        rec, sample, refs = cpu_baseline_slices(net, path, info.flops_per_slice, info.n_slices)
        got = np.array([complex(single.contract(s, 1)[0]) for s in sample])
        rms = float(np.sqrt(np.mean(np.abs(refs) ** 2)))
        rel = np.abs(got - refs) / np.abs(refs)
        res["error_vs_oracle"].update({
            "sampled_slices": len(sample), "median_rel": float(np.median(rel)), "max_rel": float(rel.max()),
            "max_abs_over_rms_amplitude": float(np.max(np.abs(got - refs)) / rms),
            "note": "per-slice amplitudes are Porter-Thomas distributed: small slices lose relative digits to "
                    "float32 cancellation, so errors are bounded against the rms amplitude (1e-5)"})
        res["cpu_baseline"] = rec
    single.close()
    plan.close()
    tn.close()
    ctx.close()
    del arena
    torch.cuda.empty_cache()
    return res


def bench_circuit40(args):
    """Sliced 40-qubit circuit (5x8 grid, depth 12, 16 sliced labels = 65,536
    slices): the slices run as a batch dimension of every step, summed in FP64."""
    rec = circuit40_record(args, args.steps, args.warmup, not args.no_cpu and not args.counters)
    if args.counters:
        print(json.dumps(rec), flush=True)
        return
    res = {"metric": "complex TFLOP/s of path execution (% MFMA peak) + p50/p99 request latency",
           "value": rec.pop("value"), "unit": rec.pop("unit"), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": rec.pop("ms_per_run"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": rec.pop("dtype"), "data": "synthetic",
           "config": rec}
    if "cpu_baseline" in rec:
        res["cpu_baseline"] = rec.pop("cpu_baseline")
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
    forms = [(prec, form)]
    if not args.no_forms and args.form == "4M" and args.prec == "c64":
        forms += [(tnc.PREC_C64, tnc.GEMM_3M), (tnc.PREC_BF16X3, tnc.GEMM_4M), (tnc.PREC_BF16X3, tnc.GEMM_3M)]
    for net, path in ((net_a, path_a), (net_b, path_b)):
        tn = tnc.Network(hctx, net.labels, net.extents, net.open)
        for fp, ff in forms:   # split precision also holds its operands' bf16 planes
            p = tnc.Plan(tn, path.pairs, (), fp, ff)
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
                   "path_roofline_frac": round((path_roofline_s(tnc, plan_a, split=prec == tnc.PREC_BF16X3,
                                                                three_m=form == tnc.GEMM_3M)
                                                + path_roofline_s(tnc, plan_b, split=prec == tnc.PREC_BF16X3,
                                                                  three_m=form == tnc.GEMM_3M))
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
                    "permute_gbs": round(perm_gbs, 1) if perm_gbs else None,
                    "permute_frac_of_hbm_peak": round(perm_gbs / PEAK_HBM, 4) if perm_gbs else None,
                    "batch_gemm_ms": round(bgemm_ms / max(bgemm_n, 1), 3),
                    "batch_gemm_tflops": round(plan_b.info.flops_per_slice / (bgemm_ms / max(bgemm_n, 1) / 1e3)
                                               / 1e12, 3) if bgemm_n else None},
    }
    # result rows kept for the comparison with the CPU oracle's sample: the
    # first 1/16 of pair30's rows (leading four M labels 0) and the first
    # four batch entries
    rows_a = plan_a.info.n_result // 16
    rows_b = plan_b.info.n_result // 16
    kept = {"4M" if prec == tnc.PREC_C64 and form == tnc.GEMM_4M else args.form:
            (out_a[:rows_a].cpu().numpy(), out_b[:rows_b].cpu().numpy())}
    if not args.no_forms and args.form == "4M" and args.prec == "c64":
        # the same step in the other GEMM forms (same inputs, same arena)
        res["other_forms"] = {}
        for name, fprec, fform, fpeak in (("3M", tnc.PREC_C64, tnc.GEMM_3M, PEAK_FP32_MFMA),
                                          ("bf16x3", tnc.PREC_BF16X3, tnc.GEMM_4M, PEAK_BF16_MFMA / 3),
                                          ("bf16x3_3M", tnc.PREC_BF16X3, tnc.GEMM_3M, PEAK_BF16_MFMA / 3)):
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
            gt = plan_a.info.flops_per_slice / g_s / 1e12
            # executed MFMA work against its own peak: the 3M forms execute
            # 6 of the 8 FLOPs per complex MAC, split-bf16x3 three bf16
            # products per real product (peak / 3 in the 8-FLOP convention)
            executed = gt * (6 / 8 if fform == tnc.GEMM_3M else 1.0) / fpeak
            res["other_forms"][name] = {
                "tflops": round(flops_step / fdt / 1e12, 3), "ms_per_step": round(fdt * 1e3, 3),
                "gemm_tflops": round(gt, 3), "gemm_frac_of_executed_mfma_peak": round(executed, 4),
                # the 8-FLOP complex convention against the form's precision
                # peak (FP32 MFMA, or bf16 MFMA / 3 for split precision)
                "gemm_frac_of_peak_8flop": round(gt / fpeak, 4),
                "variant": tnc.tnc_plan_get_step(pa.handle, 0).variant,
                "presplit": bool(tnc.tnc_plan_get_step(pa.handle, 0).presplit)}
            kept[name] = (out_a[:rows_a].cpu().numpy(), out_b[:rows_b].cpu().numpy())
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
    plan_a.close()
    plan_b.close()
    tn_a.close()
    tn_b.close()
    ctx.close()
    del arena, out_a, out_b
    torch.cuda.empty_cache()
    if not args.no_configs:
        res["configs"] = {}
        log("config record: circuit12")
        res["configs"]["circuit12"] = record_circuit12()
        log("config record: grid8")
        res["configs"]["grid8"] = record_grid8()
        log("config record: circuit40")
        res["configs"]["circuit40"] = circuit40_record(args, 2, 1, not args.no_cpu)
    if not args.no_serve:
        res["latency"] = serving_leg(args)
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample)")
        rec, ref_rows, ref_batch = cpu_baseline(net_a, path_a, net_b, path_b)
        res["cpu_baseline"] = rec
        res["error_vs_oracle"] = {"sample": "the CPU baseline's sample: pair30 rows with the leading four M labels "
                                            "0 (1/16 of the result) and the first 4 of 64 batch entries",
                                  "metric": "relative Frobenius error, and max |error| / max |ref|"}
        for name, (ga, gb) in kept.items():
            ea, ea_max = rel_err(ga, ref_rows)
            eb, eb_max = rel_err(gb[:ref_batch.size], ref_batch)
            res["error_vs_oracle"][name] = {"pair30": [ea, ea_max], "pair_batch": [eb, eb_max]}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
