"""Pins of the oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a brute
force state-vector simulation, closed forms, library routines on special
cases, order independence (paper Sec. II-B), slicing exactness (Sec. II-C),
the worked reordering example (Fig. 3), the cost example of Sec. II-B/II-E.
"""
import json
import os

import numpy as np
import pytest

from oracle import contract as oc
from oracle import costs as ocost
from oracle import reorder as orr
from oracle import split as osp
from oracle import statevector as osv
from workloads import configs
from workloads.circuits import Circuit, circuit_network, haar_unitary, random_circuit
from workloads.grids import constant_grid_network, product_grid_network, random_grid_network
from workloads.network import Network, Path
from workloads.pairs import pair_network
from workloads.paths import greedy_path, greedy_slice, random_greedy_path


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ---------------------------------------------------------------- statevector
def test_statevector_bit_order_single_x():
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    psi = osv.run(3, [((0,), x)])
    assert psi[1, 0, 0] == 1 and np.sum(np.abs(psi) ** 2) == 1
    # qubit 0 is the most significant bit of the flat index
    assert np.flatnonzero(psi.ravel())[0] == 4


def test_statevector_two_qubit_row_index():
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    cnot = np.eye(4, dtype=np.complex128)[[0, 1, 3, 2]]  # row 2*o1+o2, control q1
    psi = osv.run(2, [((0,), x), ((0, 1), cnot)])
    assert psi[1, 1] == 1
    psi = osv.run(2, [((1,), x), ((0, 1), cnot)])
    assert psi[0, 1] == 1


def test_haar_unitary_is_unitary():
    rng = np.random.Generator(np.random.PCG64(7))
    for d in (2, 4):
        u = haar_unitary(rng, d)
        assert np.allclose(u @ u.conj().T, np.eye(d), atol=1e-13)


# ----------------------------------------------------- contraction vs circuits
def test_circuit12_amplitude_matches_statevector():
    circ = configs.circuit12_circuit()
    net, path = configs.circuit12()
    amp = oc.contract(net, path, leaves=net.leaves)           # complex128 gates
    ref = osv.amplitude(circ.n_qubits, circ.gates, circ.bitstring)
    assert abs(amp - ref) <= 1e-12 * abs(ref)


def test_circuit12_all_amplitudes_and_unitarity():
    circ = configs.circuit12_circuit()
    net = circuit_network(circ, open_qubits=range(circ.n_qubits))
    path = greedy_path(net)
    amps = oc.contract(net, path, leaves=net.leaves)
    ref = osv.run(circ.n_qubits, circ.gates)
    assert amps.shape == (2,) * 12
    assert rel(amps, ref) <= 1e-12
    assert abs(np.sum(np.abs(amps) ** 2) - 1.0) <= 1e-12


def test_batched_bitstrings_match_the_state_vector():
    """A batch label shared by all projector leaves (one network, B
    amplitudes) gives the state vector's entries at the B bitstrings."""
    from workloads.circuits import circuit_network_batched
    circ = configs.circuit12_circuit()
    rng = np.random.Generator(np.random.PCG64(3))
    bits = rng.integers(0, 2, size=(16, circ.n_qubits))
    net = circuit_network_batched(circ, bits)
    amps = oc.contract(net, greedy_path(net), leaves=net.leaves)
    sv = osv.run(circ.n_qubits, circ.gates)
    ref = np.array([sv[tuple(b)] for b in bits])
    assert amps.shape == (16,)
    assert rel(amps, ref) <= 1e-12


def test_order_independence_circuit_and_grid():
    net, p1 = configs.circuit12()
    p2 = random_greedy_path(net, seed=3)
    assert not np.array_equal(p1.pairs, p2.pairs)
    a1 = oc.contract(net, p1)
    a2 = oc.contract(net, p2)
    assert abs(a1 - a2) <= 1e-12 * abs(a1)
    g = random_grid_network(4, 4, 3, seed=11)
    q1, q2 = greedy_path(g), random_greedy_path(g, seed=5)
    z1, z2 = oc.contract(g, q1), oc.contract(g, q2)
    assert abs(z1 - z2) <= 1e-12 * abs(z1)


def test_slicing_is_exact():
    net, p = configs.circuit12()
    sl = greedy_slice(net, p.pairs, n_sliced=3)
    assert len(sl) == 3
    full = oc.contract(net, p)
    parts = oc.contract(net, Path(p.pairs, sl))
    assert abs(full - parts) <= 1e-12 * abs(full)
    # a sliced sum over an open network too
    circ = configs.circuit12_circuit()
    net2 = circuit_network(circ, open_qubits=(0, 5))
    p2 = greedy_path(net2)
    sl2 = greedy_slice(net2, p2.pairs, n_sliced=2)
    assert rel(oc.contract(net2, Path(p2.pairs, sl2)), oc.contract(net2, p2)) <= 1e-12


# ------------------------------------------------------------------- grids
def test_constant_grid_is_one():
    for rows, cols, bond in ((3, 3, 2), (4, 5, 3), (8, 8, 4)):
        net = constant_grid_network(rows, cols, bond)
        z = oc.contract(net, greedy_path(net), leaves=net.leaves)
        assert abs(z - 1.0) <= 1e-12


def test_product_state_grid_closed_form():
    net, vecs = product_grid_network(5, 6, 3, seed=9)
    owners = {}
    for t, lab in enumerate(net.labels):
        for l in lab:
            owners.setdefault(l, []).append(t)
    expected = 1.0 + 0j
    for l, (s, t) in owners.items():
        expected *= np.sum(vecs[(s, l)] * vecs[(t, l)])
    z = oc.contract(net, greedy_path(net), leaves=net.leaves)
    assert abs(z - expected) <= 1e-12 * abs(expected)


def test_tiny_network_matches_single_einsum():
    """Brute force: one numpy.einsum over all labels at once."""
    net = random_grid_network(3, 3, 2, seed=4)
    letters = "abcdefghijklmnopqrstuvwxyz"
    spec = ",".join("".join(letters[l] for l in lab) for lab in net.labels) + "->"
    ref = np.einsum(spec, *net.leaves)
    z = oc.contract(net, greedy_path(net), leaves=net.leaves)
    assert abs(z - ref) <= 1e-12 * abs(ref)
    # with open labels
    circ = random_circuit(2, 2, 3, seed=2)
    net = circuit_network(circ, open_qubits=(2, 0))
    spec = ",".join("".join(letters[l] for l in lab) for lab in net.labels) + "->" + \
        "".join(letters[l] for l in net.open)
    ref = np.einsum(spec, *net.leaves)
    z = oc.contract(net, greedy_path(net), leaves=net.leaves)
    assert rel(z, ref) <= 1e-12


def test_batch_pair_matches_per_batch_matmul():
    net, p = pair_network(3, 4, 2, seed=5, batch=5)
    a, b = net.leaves
    la, lb = net.labels
    z = net.open[0]
    M, K, N = list(range(3)), list(range(3, 7)), list(range(7, 9))
    A = np.transpose(a, [la.index(l) for l in [z] + M + K]).reshape(5, 8, 16).astype(np.complex128)
    B = np.transpose(b, [lb.index(l) for l in [z] + N + K]).reshape(5, 4, 16).astype(np.complex128)
    ref = np.stack([A[i] @ B[i].T for i in range(5)]).reshape((5,) + (2,) * 5)
    got = oc.contract(net, p)
    assert rel(got, ref) <= 1e-13


def test_validation_rejects_non_networks():
    with pytest.raises(ValueError):
        oc.label_kinds([(0, 1), (1, 2), (1, 3)], (0, 2, 3))   # closed hyperedge
    with pytest.raises(ValueError):
        oc.label_kinds([(0, 1), (1,)], ())                    # dangling closed label
    with pytest.raises(ValueError):
        oc.check_path(3, np.array([[0, 1], [0, 2]]))          # id used twice
    with pytest.raises(ValueError):
        oc.check_path(3, np.array([[0, 1]]))                  # not a full tree


# ----------------------------------------------- planted mistakes are caught
def test_planted_mistakes_fail_the_pins(monkeypatch):
    circ = configs.circuit12_circuit()
    net = circuit_network(circ, open_qubits=range(circ.n_qubits))
    path = greedy_path(net)
    ref = osv.run(circ.n_qubits, circ.gates)
    good = oc.pairwise

    def conj_one(x, la, y, lb, keep):          # a conjugated operand
        return good(np.conj(x), la, y, lb, keep)

    def drop_one_term(x, la, y, lb, keep):     # one term of a sum left out
        summed = [l for l in la if l in lb and l not in keep]
        if not summed:
            return good(x, la, y, lb, keep)
        ax = la.index(summed[0])
        x2 = x.copy()
        idx = [slice(None)] * x.ndim
        idx[ax] = 0
        x2[tuple(idx)] = 0
        return good(x2, la, y, lb, keep)

    def transposed(x, la, y, lb, keep):        # labels attached to the wrong axes
        z, lz = good(x, la, y, lb, keep)
        return z, lz[::-1] if len(lz) > 1 and len(set(z.shape)) == 1 else lz

    for bad in (conj_one, drop_one_term, transposed):
        got = oc.contract_tree(net.leaves, net.labels, net.open, path.pairs, step=bad)
        assert rel(got, ref) > 1e-6, bad.__name__


# ---------------------------------------------------------------- reordering
def _fig3(golden_dir):
    d = json.load(open(os.path.join(golden_dir, "fig3_reorder.json")))
    L = d["labels"]
    lab = lambda s: tuple(L[c] for c in s)
    names = ["I1", "I2", "I3"]
    labels = [lab(d["leaves"][n]) for n in names]
    ids = {"I1": 0, "I2": 1, "I3": 2, "I4": 3, "I5": 4}
    pairs = np.array([[ids[a], ids[b]] for a, b in d["pairs"]])
    return d, labels, pairs, lab(d["root_order"]), ids, lab


def test_fig3_worked_example(golden_dir):
    d, labels, pairs, root, ids, lab = _fig3(golden_dir)
    target, steps = orr.reorder(labels, pairs, root)
    for name, want in d["expected"].items():
        assert tuple(target[ids[name]]) == lab(want), name
    for name, want in d["expected_split"].items():
        left, right = want.split("|")
        t = tuple(target[ids[name]])
        assert t[:len(left)] == lab(left) and t[len(left):] == lab(right)
    assert steps[0]["natural"] is (not d["expected_interleaved_output"]["step1"])
    assert steps[1]["natural"] is (not d["expected_interleaved_output"]["step2"])
    assert tuple(target[ids["I5"]]) == root


def _random_tree_network(rng, n_leaves, n_open):
    """Random binary tree with random closed labels between random leaf pairs."""
    labels = [[] for _ in range(n_leaves)]
    nxt = 0
    for t in range(1, n_leaves):          # spanning tree keeps it connected
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
    leaves = [(rng.standard_normal(tuple(ext[l] for l in lab)) + 0j) for lab in labels]
    return Network(leaves, labels, ext, tuple(opn))


@pytest.mark.parametrize("seed", range(12))
def test_reorder_invariants_random_trees(seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    net = _random_tree_network(rng, int(rng.integers(2, 14)), int(rng.integers(0, 4)))
    path = random_greedy_path(net, seed=seed)
    target, steps = orr.reorder(net.labels, path.pairs, net.open)
    tag = orr.lifetimes(net.labels, path.pairs, net.open)
    # every tensor holds exactly its labels; modes sorted by remaining lifetime
    for t, order in enumerate(target):
        tags = [tag[l] for l in order]
        assert all(tags[i] >= tags[i + 1] for i in range(len(tags) - 1)), (t, order, tags)
    for st in steps:
        A, B, C = target[st["A"]], target[st["B"]], target[st["C"]]
        K = st["K"]
        assert A == [l for l in C if l in A] + K and B == [l for l in C if l in B] + K
        assert sorted(C) == sorted(st["M"] + st["N"] + st["H"])
        assert K == sorted(K)
    # determinism
    assert orr.reorder(net.labels, path.pairs, net.open) == (target, steps)
    # result unchanged when every leaf is stored in its target order
    leaves2 = [np.transpose(x, [lab.index(l) for l in target[t]])
               for t, (x, lab) in enumerate(zip(net.leaves, net.labels))]
    net2 = Network(leaves2, [tuple(target[t]) for t in range(net.n_leaves)], net.extents, net.open)
    a = oc.contract(net, path, leaves=net.leaves)
    b = oc.contract(net2, path, leaves=net2.leaves)
    assert rel(b, a) <= 1e-12 or np.allclose(a, b, atol=1e-12)


# --------------------------------------------------------------------- costs
def test_cost_example(golden_dir):
    d = json.load(open(os.path.join(golden_dir, "cost_example.json")))
    lhs, out = d["einsum"].split("->")
    a, b = lhs.split(",")
    code = {c: i for i, c in enumerate(sorted(set(a + b)))}
    labels = [tuple(code[c] for c in a), tuple(code[c] for c in b)]
    open_labels = tuple(code[c] for c in out)
    ext = np.full(len(code), d["extent"], dtype=np.int64)
    target, steps = orr.reorder(labels, np.array([[0, 1]]), open_labels)
    c = ocost.step_costs(steps, target, ext)[0]
    for key in ("m", "n", "k", "Ct", "Cs", "Cm"):
        assert c[key] == d[key], key
    assert ocost.path_totals([c])["flops"] == d["flops"]


def test_cost_counts_match_brute_force_multiply_adds():
    """C_t = number of scalar multiply-adds a naive loop performs."""
    rng = np.random.Generator(np.random.PCG64(3))
    net = _random_tree_network(rng, 6, 2)
    path = greedy_path(net)
    target, steps = orr.reorder(net.labels, path.pairs, net.open)
    for st, c in zip(steps, ocost.step_costs(steps, target, net.extents)):
        allx = set(target[st["A"]]) | set(target[st["B"]])
        n = 1
        for l in allx:
            n *= int(net.extents[l])
        assert c["Ct"] == n


# --------------------------------------------------------------------- split
def test_bf16_rne_known_values():
    f = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 0.0], dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 0.0], dtype=np.float32)
    assert np.array_equal(osp.bf16_rne(f), want)


def test_bf16_rne_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(1))
    x = (rng.standard_normal(100000) * 10.0 ** rng.integers(-30, 30, 100000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(osp.bf16_rne(x), ref)


def test_split_error_bounds():
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.standard_normal(20000).astype(np.float32)
    y = rng.standard_normal(20000).astype(np.float32)
    xh, xl = osp.split(x)
    assert np.all(np.abs(x - (xh + xl)) <= 2.0 ** -16 * np.abs(x))
    yh, yl = osp.split(y)
    p3 = xh * yh + xh * yl + xl * yh
    exact = x.astype(np.float64) * y.astype(np.float64)
    assert np.all(np.abs(p3 - exact) <= 3 * 2.0 ** -16 * np.abs(exact) + 1e-300)


def _small_integer_pair(rng, shape_a, shape_b):
    """Complex operands with integer parts in [-100, 100]: every part, every
    float32 sum of two parts and every product sum below is exact in bf16
    hi alone (lo = 0) and in float64."""
    a = rng.integers(-100, 101, shape_a + (2,)).astype(np.float64)
    b = rng.integers(-100, 101, shape_b + (2,)).astype(np.float64)
    return a[..., 0] + 1j * a[..., 1], b[..., 0] + 1j * b[..., 1]


def test_split_3m_step_is_exact_on_bf16_exact_integers():
    """3M split form: on operands that bf16 holds exactly the dropped
    lo * lo term is zero, so the emulation must equal the exact complex
    product element for element (a dropped or mis-signed T term, a wrong
    sum plane or swapped re/im fails)."""
    rng = np.random.Generator(np.random.PCG64(31))
    x, y = _small_integer_pair(rng, (6, 20), (5, 20))
    got, lz = osp.split_step_3m(x, (0, 2), y, (1, 2), (0, 1))
    assert tuple(lz) == (0, 1)
    assert np.array_equal(got, x @ y.T)


def test_split_3m_step_equals_4m_on_real_operands():
    """With zero imaginary parts T2 = 0 and T3 = T1 exactly, so the 3M
    split step is the 4M split step (already pinned above) bit for bit."""
    rng = np.random.Generator(np.random.PCG64(32))
    x = rng.standard_normal((7, 33)).astype(np.float32).astype(np.complex128)
    y = rng.standard_normal((9, 33)).astype(np.float32).astype(np.complex128)
    m3, _ = osp.split_step_3m(x, (0, 2), y, (1, 2), (0, 1))
    m4, _ = osp.split_step(x, (0, 2), y, (1, 2), (0, 1))
    assert np.array_equal(m3, m4)
    assert np.all(m3.imag == 0)


def test_split_3m_step_within_its_bound():
    """Random float32 operands: each element of the 3M split step lies
    within 3 * 2^-16 of the magnitudes of its three real products (plus
    the complex64 rounding) of the exact product, and the lo terms matter
    (hi products alone miss by far more)."""
    rng = np.random.Generator(np.random.PCG64(33))
    def c32(shape):
        return (rng.standard_normal(shape).astype(np.float32)
                + 1j * rng.standard_normal(shape).astype(np.float32)).astype(np.complex128)
    x, y = c32((8, 64)), c32((6, 64))
    got, _ = osp.split_step_3m(x, (0, 2), y, (1, 2), (0, 1))
    exact = x @ y.T
    ar, ai, br, bi = np.abs(x.real), np.abs(x.imag), np.abs(y.real), np.abs(y.imag)
    t1, t2 = ar @ br.T, ai @ bi.T
    t3 = (ar + ai) @ (br + bi).T
    bound_re = 3 * 2.0 ** -16 * (t1 + t2) + 2.0 ** -23 * np.abs(exact.real)
    bound_im = 3 * 2.0 ** -16 * (t1 + t2 + t3) * (1 + 2.0 ** -20) + 2.0 ** -23 * np.abs(exact.imag)
    assert np.all(np.abs(got.real - exact.real) <= bound_re)
    assert np.all(np.abs(got.imag - exact.imag) <= bound_im)
    hi_only = osp.bf16_rne(x.real.astype(np.float32)).astype(np.float64) @ osp.bf16_rne(
        y.real.astype(np.float32)).astype(np.float64).T
    assert np.max(np.abs(hi_only - x.real @ y.real.T)) > 4 * np.max(3 * 2.0 ** -16 * t1)


def test_split_emulation_tracks_exact_path():
    net, p = configs.circuit12()
    exact = oc.contract(net, p)
    emu = oc.contract(net, p, step=osp.split_step)
    c64 = oc.contract(net, p, step=osp.c64_step)
    assert abs(c64 - exact) <= 1e-5 * abs(exact)
    assert 1e-9 < abs(emu - exact) / abs(exact) <= 1e-3
    emu3 = oc.contract(net, p, step=osp.split_step_3m)
    assert 1e-9 < abs(emu3 - exact) / abs(exact) <= 1e-3
    assert emu3 != emu   # a different sequence of roundings
