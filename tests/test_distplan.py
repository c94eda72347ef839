"""Distribution planning (paper Sec. IV-B): the library's DP against the
oracle's exhaustive enumeration of keep/redistribute schedules, plus the
cost formulas on a hand-computed example."""
import json
import os

import numpy as np
import pytest

from oracle import distplan as od
from paper_2606_01852_amd import tnc

HW = dict(B_dev=8e12, F_dev=157.3e12, B_net=448e9, lat=10e-6)


def test_cost_formulas_hand_example(golden_dir):
    d = json.load(open(os.path.join(golden_dir, "dist_cost_example.json")))
    for case in d["prefix"]:
        ext = case["ext"]
        ext = {int(k): v for k, v in ext.items()} if isinstance(ext, dict) else dict(enumerate(ext))
        assert list(od.prefix_modes(case["order"], ext, case["P"])) == case["expect"]
    c = d["comm"]
    eq = dict(order=c["order"], ext={l: 2 for l in c["order"]}, c=c["c"])
    got = od.t_comm(eq, c["P"], dict(B_net=c["B_net"], lat=c["lat"]), tuple(c["old"]), tuple(c["new"]))
    assert abs(got - c["expect"]) <= 1e-15


def test_gemm_and_gather_terms_hand_example(golden_dir):
    """Eq. (6) per-device GEMM time (chain operand and output split P ways,
    the other operand whole on every device) and the chain-end gather, on
    hand-computed values: a replicated operand divided by P, or a gather
    without its (P - 1) / P factor, misses them."""
    d = json.load(open(os.path.join(golden_dir, "dist_cost_example.json")))
    for g in d["gemm"]:
        eq = dict(a=g["a"], b=g["b"], c=g["c"], ops=g["ops"])
        got = od.t_gemm(eq, g["P"], dict(B_dev=g["B_dev"], F_dev=g["F_dev"]))
        assert got == pytest.approx(g["expect"], rel=1e-12)
    g = d["gather"]
    assert od.t_gather(dict(c=g["c"]), g["P"], dict(B_net=g["B_net"])) == pytest.approx(g["expect"], rel=1e-12)


def test_chain_schedule_hand_example(golden_dir):
    """A three-equation chain whose every term was computed by hand (Eq. (4)
    prefixes, Eq. (6) per equation, one forced redistribution under Eq. (7),
    the final gather): the oracle's enumeration and the library's DP both
    reach exactly the hand-computed optimum and schedule."""
    c = json.load(open(os.path.join(golden_dir, "dist_cost_example.json")))["chain"]
    hw = dict(B_dev=c["B_dev"], F_dev=c["F_dev"], B_net=c["B_net"], lat=c["lat"])
    ext = np.full(c["n_labels"], 2, dtype=np.int64)
    labels = [tuple(x) for x in c["labels"]]
    pairs = np.array(c["pairs"], dtype=np.int32)
    chains = od.use_chains(labels, pairs, tuple(c["open"]), ext, c["large_bytes"])
    assert len(chains) == 1 and [e["step"] for e in chains[0]] == [0, 1, 2]
    for e, tg in zip(chains[0], c["t_gemm"]):
        assert od.t_gemm(e, c["P"], hw) == pytest.approx(tg, rel=1e-12)
    best, bits = od.brute_force(chains[0], c["P"], hw)
    assert best == pytest.approx(c["total"], rel=1e-12) and list(bits) == c["redist"]
    assert od.evaluate(chains[0], c["P"], hw, [False, False]) is None   # keeping (0, 1) into eq2 is forbidden
    plan = tnc.Plan(tnc.Network(tnc.Context(-1), labels, ext, tuple(c["open"])), pairs)
    steps, total, moved = tnc.tnc_plan_distribute(plan.handle, c["P"], c["large_bytes"], hw["B_dev"], hw["F_dev"],
                                                  hw["B_net"], hw["lat"])
    assert [s.state for s in steps] == c["states"]
    assert [s.t_gemm_s for s in steps] == pytest.approx(c["t_gemm"], rel=1e-12)
    assert steps[1].t_comm_s == pytest.approx(c["t_comm"], rel=1e-12)
    assert total == pytest.approx(c["total"], rel=1e-12)
    assert moved == pytest.approx(c["moved"], rel=1e-12)


def caterpillar(rng, n_side, n_main=8, max_new=3, max_sum=3):
    """A main tensor absorbing side tensors one by one (all extents 2): each
    side tensor sums some current modes of the main tensor and adds new
    ones, so the main tensor's size rises and falls along the chain."""
    nxt = n_main
    main = list(range(n_main))
    labels = [tuple(main)]
    for _ in range(n_side):
        k = int(rng.integers(0, min(max_sum, len(main) - 2) + 1))
        summed = [int(x) for x in rng.choice(main, k, replace=False)] if k else []
        new = list(range(nxt, nxt + int(rng.integers(0, max_new + 1))))
        nxt += len(new)
        labels.append(tuple(int(x) for x in rng.permutation(summed + new)))
        main = [l for l in main if l not in summed] + new
    n = len(labels)
    pairs = [[0, 1]] + [[n + i, i + 2] for i in range(n_side - 1)]
    return labels, np.array(pairs, dtype=np.int32), tuple(main), np.full(nxt, 2, dtype=np.int64)


@pytest.mark.parametrize("seed", range(16))
def test_dp_matches_exhaustive_enumeration(seed):
    rng = np.random.Generator(np.random.PCG64(900 + seed))
    labels, pairs, opn, ext = caterpillar(rng, int(rng.integers(4, 12)))
    P = int(rng.choice([2, 4, 8, 16]))
    hw = dict(B_dev=float(rng.choice([1e9, 8e12])), F_dev=157.3e12, B_net=float(rng.choice([1e8, 448e9])),
              lat=float(rng.choice([0.0, 1e-5, 1e-3])))
    large = float(8 * 2 ** int(rng.integers(4, 9)))
    ctx = tnc.Context(-1)
    tn = tnc.Network(ctx, labels, ext, opn)
    plan = tnc.Plan(tn, pairs)
    steps, total, moved = tnc.tnc_plan_distribute(plan.handle, P, large, hw["B_dev"], hw["F_dev"],
                                                  hw["B_net"], hw["lat"])
    chains = od.use_chains(labels, pairs, opn, ext, large)
    expect_total = 0.0
    by_chain = {}
    for s in steps:
        by_chain.setdefault(s.chain, []).append(s)
    feasible = [c for c in chains if od.brute_force(c, P, hw) is not None]
    assert len(by_chain) == len(feasible)
    for (cid, recs), chain in zip(sorted(by_chain.items()), feasible):
        assert [r.step for r in recs] == [e["step"] for e in chain]
        best, _ = od.brute_force(chain, P, hw)
        expect_total += best
        # the library's schedule is feasible and optimal under the oracle's costs
        redist = [r.state == 2 for r in recs[1:]]
        mine = od.evaluate(chain, P, hw, redist)
        assert mine is not None and mine == pytest.approx(best, rel=1e-9)
        assert recs[0].state == 0
        # distributed modes follow Eq. (4) wherever they are (re)chosen
        for r, e in zip(recs, chain):
            if r.state in (0, 2):
                assert tuple(r.dist[:r.n_dist]) == od.prefix_modes(e["order"], e["ext"], P)
    assert total == pytest.approx(expect_total, rel=1e-9)


def test_redistribution_goes_to_the_size_valley():
    """Fig. 5's behaviour on a made-up chain: the modes distributed first are
    summed at the end, so a redistribution is unavoidable; the tensor is
    large (2^13), then small (2^7, the valley), then large again (2^12) before
    those modes are summed.  The cheapest schedule redistributes in the
    valley, not on either plateau or at the forced point."""
    leaf0 = tuple(range(10))                      # modes 0..9
    sides = [(9,),                                # step 0: sum 9          -> 2^9
             (10, 11, 12, 13),                    # step 1: add 4 (open)   -> 2^13
             (3, 4, 5, 6, 7, 8),                  # step 2: sum 6          -> 2^7
             (14, 15, 16, 17, 18),                # step 3: add 5 (open)   -> 2^12
             (0, 1, 2)]                           # step 4: sum 0, 1, 2    -> 2^9
    labels = [leaf0] + sides
    n = len(labels)
    pairs = np.array([[0, 1]] + [[n + i, i + 2] for i in range(len(sides) - 1)], dtype=np.int32)
    ext = np.full(19, 2, dtype=np.int64)
    opn = tuple(range(10, 19))
    plan = tnc.Plan(tnc.Network(tnc.Context(-1), labels, ext, opn), pairs)
    hw = dict(B_dev=8e12, F_dev=157.3e12, B_net=448e9, lat=10e-6)
    steps, total, moved = tnc.tnc_plan_distribute(plan.handle, 8, 8 * 2 ** 6, hw["B_dev"], hw["F_dev"],
                                                  hw["B_net"], hw["lat"])
    assert [s.step for s in steps] == [0, 1, 2, 3, 4]
    assert [s.out_bytes for s in steps] == [8 * 2 ** 9, 8 * 2 ** 13, 8 * 2 ** 7, 8 * 2 ** 12, 8 * 2 ** 9]
    assert tuple(steps[0].dist[:steps[0].n_dist]) == (0, 1, 2) or set(steps[0].dist[:3]) == {0, 1, 2}
    assert [s.state for s in steps] == [0, 1, 2, 1, 1]          # redistribute at the valley only
    assert set(steps[2].dist[:steps[2].n_dist]) <= set(range(10, 14))
    assert moved == pytest.approx(8 * 2 ** 7 * 7 / 8)
    chains = od.use_chains(labels, pairs, opn, ext, 8 * 2 ** 6)
    best = od.brute_force(chains[0], 8, hw)
    assert total == pytest.approx(best[0], rel=1e-12) and list(best[1]) == [False, True, False, False]


def test_planner_on_a_circuit_workload():
    """The 40-qubit circuit (no slicing) planned for 8 MI355X-like devices:
    every use-chain of at most 12 equations gets the exhaustive optimum, and
    every equation keeps or takes an Eq. (4) prefix of its output's modes."""
    from workloads import configs
    net, path = configs.circuit40(n_sliced=0)
    plan = tnc.Plan(tnc.Network(tnc.Context(-1), net.labels, net.extents, net.open), path.pairs)
    hw = dict(B_dev=5.4e12, F_dev=140e12, B_net=7 * 153e9, lat=10e-6)
    large = 8.0 * 2 ** 24
    steps, total, moved = tnc.tnc_plan_distribute(plan.handle, 8, large, hw["B_dev"], hw["F_dev"],
                                                  hw["B_net"], hw["lat"])
    assert steps and total > 0 and moved >= 0
    chains = od.use_chains(net.labels, path.pairs, net.open, net.extents, large)
    by_chain = {}
    for s in steps:
        by_chain.setdefault(s.chain, []).append(s)
    feasible = [c for c in chains if od.prefix_modes(c[0]["order"], c[0]["ext"], 8)]
    checked = 0
    for (cid, recs), chain in zip(sorted(by_chain.items()), feasible):
        assert [r.step for r in recs] == [e["step"] for e in chain]
        if len(chain) <= 12:
            best = od.brute_force(chain, 8, hw)
            mine = od.evaluate(chain, 8, hw, [r.state == 2 for r in recs[1:]])
            assert best is not None and mine == pytest.approx(best[0], rel=1e-9)
            checked += 1
    print(f"{len(by_chain)} chains, {len(steps)} equations, {checked} checked exhaustively; "
          f"modelled {total:.3e} s, {moved / 1e9:.2f} GB redistributed")
    assert checked >= 1
