"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test fixes the oracle (or the QPD data fed to it) against something
independent: a physical statevector of the uncut circuit, a channel
identity, a textbook routine, a closed form, brute force, or the numbers
the paper prints for its worked example.
"""

import json
import os

import itertools

import numpy as np
import pytest

import oracle
from workloads import configs, qpd
from oracle import statevector as sv
import circuit_nets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- QPD data

def _rand_rho(rng, n):
    d = 2 ** n
    a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    rho = a @ a.conj().T
    return rho / np.trace(rho)


def test_pauli_wire_identity():
    """rho = sum_P w_P Tr(P rho) P with w = (1/2,1/2,1/2,1/2) (wire cut)."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = _rand_rho(rng, 1)
        rec = sum(w * np.trace(sv.PAULI[p] @ rho) * sv.PAULI[p]
                  for w, p in zip(qpd.WIRE_PAULI, qpd.PAULI_ORDER))
        assert np.abs(rec - rho).max() < 1e-15


def test_cutqc_wire_tensor_identity():
    """Eq. wire-tensor: rho = sum_ab c_w[a,b] Tr(A_a rho) |B_b><B_b|."""
    rng = np.random.default_rng(2)
    for _ in range(5):
        rho = _rand_rho(rng, 1)
        rec = np.zeros((2, 2), dtype=complex)
        for a, pa in enumerate(qpd.CW_ROWS):
            for b, sb in enumerate(qpd.CW_COLS):
                v = sv.STATES[sb]
                rec += qpd.CW[a, b] * np.trace(sv.PAULI[pa] @ rho) * np.outer(v, v.conj())
        assert np.abs(rec - rho).max() < 1e-15


def _channel(name, rho2, qubit):
    """Apply a single-qubit instance operation to qubit `qubit` of a 2-qubit rho."""
    def lift(u):
        return np.kron(u, sv.I2) if qubit == 0 else np.kron(sv.I2, u)
    if name == "MZ":
        p0 = lift(np.diag([1.0, 0.0]).astype(complex))
        p1 = lift(np.diag([0.0, 1.0]).astype(complex))
        return p0 @ rho2 @ p0 - p1 @ rho2 @ p1
    u = lift({"S": sv.S, "Sdg": sv.SDG, "Z": sv.Z, "I": sv.I2}[name])
    return u @ rho2 @ u.conj().T


def test_cz_gate_cut_channel_identity():
    """CZ rho CZ = sum_i c_i (A_i (x) B_i)(rho) over the six instances."""
    cz = np.diag([1.0, 1.0, 1.0, -1.0]).astype(complex)
    rng = np.random.default_rng(3)
    assert abs(qpd.CZ_COEFFS.sum() - 1.0) < 1e-15
    assert abs(np.abs(qpd.CZ_COEFFS).sum() - 3.0) < 1e-15  # gamma = 3
    for _ in range(5):
        rho = _rand_rho(rng, 2)
        rec = np.zeros((4, 4), dtype=complex)
        for c, (a, b) in zip(qpd.CZ_COEFFS, qpd.CZ_INSTANCES):
            rec += c * _channel(b, _channel(a, rho, 0), 1)
        assert np.abs(rec - cz @ rho @ cz).max() < 1e-15


@pytest.mark.parametrize("theta", [0.0, 0.37, -1.2, np.pi / 2, 2.9, np.pi])
def test_rzz_gate_cut_channel_identity(theta):
    """RZZ(theta) rho RZZ(theta)^dag = sum_i c_i(theta) (A_i (x) B_i)(rho)."""
    u = np.diag(np.exp(-0.5j * theta * np.array([1.0, -1.0, -1.0, 1.0])))
    c = qpd.rzz_coeffs(theta)
    assert abs(c.sum() - 1.0) < 1e-15
    assert abs(np.abs(c).sum() - (1.0 + 2.0 * abs(np.sin(theta)))) < 1e-15  # gamma
    rng = np.random.default_rng(5)
    for _ in range(4):
        rho = _rand_rho(rng, 2)
        rec = np.zeros((4, 4), dtype=complex)
        for ci, (a, b) in zip(c, qpd.RZZ_INSTANCES):
            rec += ci * _channel(b, _channel(a, rho, 0), 1)
        assert np.abs(rec - u @ rho @ u.conj().T).max() < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_general_two_qubit_gate_cut_channel_identity(seed):
    """A random two-qubit gate in KAK form, cut as three rotation cuts (each
    the six RZZ instances conjugated into its Pauli axis): the 216 weighted
    instance channels sum to U rho U^dag, and gamma is the product of the
    three rotations' 1 + 2 |sin 2t|."""
    from workloads import circuits as c
    rng = np.random.default_rng(seed)
    a1, a2, b1, b2 = (c.random_u2(rng) for _ in range(4))
    t = rng.uniform(-np.pi / 2, np.pi / 2, size=3)
    u = c.kak_gate(a1, a2, b1, b2, t)
    assert np.abs(u @ u.conj().T - np.eye(4)).max() < 1e-14

    def conj_channel(name, v, rho2, qubit):
        lift = (lambda m: np.kron(m, sv.I2)) if qubit == 0 else (lambda m: np.kron(sv.I2, m))
        vv = lift(v)
        return vv @ _channel(name, vv.conj().T @ rho2 @ vv, qubit) @ vv.conj().T

    gamma = 1.0
    for tk in t:
        cf = qpd.kak_coeffs(tk)
        assert abs(cf.sum() - 1.0) < 1e-15
        gamma *= np.abs(cf).sum()
    assert abs(gamma - np.prod(1.0 + 2.0 * np.abs(np.sin(2.0 * t)))) < 1e-13
    for _ in range(3):
        rho = _rand_rho(rng, 2)
        b = np.kron(b1, b2)
        start = b @ rho @ b.conj().T
        rec = np.zeros((4, 4), dtype=complex)
        for idx in itertools.product(range(6), repeat=3):
            r = start
            w = 1.0
            for k, (p, i) in enumerate(zip(qpd.KAK_AXES, idx)):
                w *= qpd.kak_coeffs(t[k])[i]
                left, right = qpd.RZZ_INSTANCES[i]
                r = conj_channel(right, c.KAK_V[p], conj_channel(left, c.KAK_V[p], r, 0), 1)
            rec += w * r
        a = np.kron(a1, a2)
        assert np.abs(a @ rec @ a.conj().T - u @ rho @ u.conj().T).max() < 1e-14


def test_cx_gate_cut_channel_identity():
    """CX = (I (x) H) CZ (I (x) H): the CZ instances with the target's
    operation conjugated by H reconstruct CX rho CX."""
    cx = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    h2 = np.kron(sv.I2, sv.H)
    rng = np.random.default_rng(6)
    for _ in range(4):
        rho = _rand_rho(rng, 2)
        rec = np.zeros((4, 4), dtype=complex)
        for c, (a, b) in zip(qpd.CZ_COEFFS, qpd.CZ_INSTANCES):
            rec += c * h2 @ _channel(b, _channel(a, h2 @ rho @ h2, 0), 1) @ h2
        assert np.abs(rec - cx @ rho @ cx).max() < 1e-15


# ------------------------------------------------ naive sum vs statevector

@pytest.mark.parametrize("seed", range(4))
def test_naive_equals_uncut_statevector_wire_cuts(seed):
    net = circuit_nets.cut_wires(seed)
    full = circuit_nets.cut_wires_full(seed)
    got, n_terms = oracle.naive_contract(net.tensors, net.labels, net.dims, net.out_labels)
    assert n_terms == 16
    assert abs(float(got) - full) < 1e-14
    hi, lo = oracle.ve_contract(net.tensors, net.labels, net.dims, net.out_labels)
    assert abs(float(hi) - full) < 1e-14


@pytest.mark.parametrize("gate", ["cz", "rzz", "cx", "general"])
@pytest.mark.parametrize("n_cuts", [1, 2])
def test_naive_equals_uncut_statevector_gate_cuts(n_cuts, gate):
    if gate == "general" and n_cuts == 2:
        pytest.skip("two general gates: 8^6 branch instances per side, too slow for the oracle's "
                    "statevector; covered on the GPU evaluator against the uncut circuit")
    for seed in range(3):
        net, full = circuit_nets.cut_gates(seed, n_cuts, gate=gate)
        got, _ = oracle.naive_contract(net.tensors, net.labels, net.dims, net.out_labels)
        assert abs(float(got) - full) < 1e-14


# ---------------------------------------------- textbook special cases

def test_naive_and_ve_reduce_to_matmul():
    rng = np.random.default_rng(4)
    a = rng.normal(size=(5, 7))
    b = rng.normal(size=(7, 3))
    c = rng.normal(size=7)
    labels = [[0, 1], [1, 2], [1]]
    dims = [5, 7, 3]
    ref = a @ np.diag(c) @ b
    got, _ = oracle.naive_contract([a, b, c], labels, dims, [0, 2])
    assert np.abs(got - ref).max() < 1e-13
    hi, _ = oracle.ve_contract([a, b, c], labels, dims, [0, 2])
    assert np.abs(hi - ref).max() < 1e-13
    # transposed output order
    hi, _ = oracle.ve_contract([a, b, c], labels, dims, [2, 0])
    assert np.abs(hi - ref.T).max() < 1e-13
    # a label summed out of a single tensor, and a broadcast output label
    got, _ = oracle.naive_contract([a], [[0, 1]], [5, 7], [0])
    assert np.abs(got - a.sum(axis=1)).max() < 1e-13


def _rank1_network(rng, net):
    """Replace every tensor by an outer product of per-mode vectors."""
    vecs, tensors = [], []
    for ls in net.labels:
        vs = [rng.uniform(-1, 1, size=net.dims[l]) for l in ls]
        t = np.array(1.0)
        for v in vs:
            t = np.multiply.outer(t, v)
        vecs.append(vs)
        tensors.append(t)
    # closed form: prod over labels of sum_k prod over tensors carrying it
    total = 1.0
    for l in range(len(net.dims)):
        acc = np.ones(net.dims[l])
        seen = False
        for ls, vs in zip(net.labels, vecs):
            if l in ls:
                acc = acc * vs[ls.index(l)]
                seen = True
        if seen:
            total *= acc.sum()
    return tensors, total


@pytest.mark.parametrize("maker", ["grid", "ring"])
def test_ve_rank1_closed_form_full_size(maker):
    rng = np.random.default_rng(5)
    net = configs.grid_network(0) if maker == "grid" else configs.ring_of_rings(0)
    tensors, ref = _rank1_network(rng, net)
    hi, lo = oracle.ve_contract(tensors, net.labels, net.dims, [])
    assert abs(float(hi) + float(lo) - ref) <= 1e-13 * abs(ref)


def test_naive_rank1_closed_form():
    rng = np.random.default_rng(6)
    net, _ = circuit_nets.cut_gates(0, 2)
    tensors, ref = _rank1_network(rng, net)
    got, _ = oracle.naive_contract(tensors, net.labels, net.dims, [])
    assert abs(float(got) - ref) <= 1e-14 * max(1.0, abs(ref))


def test_ve_onehot_coefficients_select_single_entries():
    """One-hot CTs collapse the network to a product of single QT entries."""
    rng = np.random.default_rng(7)
    for net in (configs.grid_network(3), configs.ring_of_rings(3)):
        pick = {}
        tensors = []
        for t, ls, kind in zip(net.tensors, net.labels, net.kinds):
            if kind == "ct":
                k = int(rng.integers(net.dims[ls[0]]))
                pick[ls[0]] = k
                e = np.zeros(net.dims[ls[0]])
                e[k] = 1.0
                tensors.append(e)
            else:
                tensors.append(t)
        ref = 1.0
        for t, ls, kind in zip(net.tensors, net.labels, net.kinds):
            if kind == "qt":
                ref *= t[tuple(pick[l] for l in ls)]
        hi, lo = oracle.ve_contract(tensors, net.labels, net.dims, [])
        assert abs(float(hi) - ref) <= 1e-15 * abs(ref) + 1e-300


# ------------------------------------------------------ brute force

def _random_small_network(rng):
    n_labels = int(rng.integers(3, 7))
    dims = [int(d) for d in rng.integers(2, 5, size=n_labels)]
    n_t = int(rng.integers(2, 6))
    labels = []
    for _ in range(n_t):
        r = int(rng.integers(1, min(4, n_labels) + 1))
        labels.append([int(x) for x in rng.choice(n_labels, size=r, replace=False)])
    used = sorted({l for ls in labels for l in ls})
    n_out = int(rng.integers(0, 3))
    out = [int(x) for x in rng.choice(used, size=min(n_out, len(used)), replace=False)]
    tensors = [rng.uniform(-1, 1, size=[dims[l] for l in ls]) for ls in labels]
    return tensors, labels, dims, out


def test_ve_equals_naive_random_networks():
    rng = np.random.default_rng(8)
    for _ in range(60):
        tensors, labels, dims, out = _random_small_network(rng)
        naive, _ = oracle.naive_contract(tensors, labels, dims, out)
        hi, lo = oracle.ve_contract(tensors, labels, dims, out)
        f64 = oracle.ve_contract(tensors, labels, dims, out, mode="f64")
        scale = max(1.0, float(np.abs(naive).max()))
        assert np.abs(hi - naive).max() <= 1e-13 * scale
        assert np.abs(f64 - naive).max() <= 1e-12 * scale
        # einsum as an independent library cross-check
        letters = "abcdefghij"
        spec = ",".join("".join(letters[l] for l in ls) for ls in labels)
        spec += "->" + "".join(letters[l] for l in out)
        assert np.abs(np.einsum(spec, *tensors) - naive).max() <= 1e-12 * scale


def test_double_double_resolves_cancellation():
    """(1e16 + 1) - 1e16 = 1 exactly; plain FP64 loses the 1."""
    u = np.array([1e16, 1.0, -1e16])
    w = np.ones(3)
    hi, lo = oracle.ve_contract([u, w], [[0], [0]], [3], [])
    assert float(hi) + float(lo) == 1.0
    assert float(oracle.ve_contract([u, w], [[0], [0]], [3], [], mode="f64")) == 0.0
    got, _ = oracle.naive_contract([u, w], [[0], [0]], [3], [])
    assert float(got) == 1.0


# ------------------------------------------------------ marginal

def test_marginal_invariants_and_matrix_form():
    net = configs.marginal_network(0, out_bits=4, n_cuts=4)
    r, n_terms = oracle.naive_contract(net.tensors, net.labels, net.dims, net.out_labels)
    assert abs(r.sum() - 1.0) < 1e-13          # sum_x R = (sum c_w)^4 = 1
    assert np.abs(r).sum() > 1.5               # signed: real cancellation
    t1 = net.tensors[0].reshape(256, -1)
    t2 = net.tensors[1].reshape(256, -1)
    c = qpd.CW
    big = np.kron(np.kron(np.kron(c, c), c), c)  # rows a1..a4, cols b1..b4
    ref = t1.T @ big @ t2
    assert np.abs(r - ref).max() < 1e-15
    hi, _ = oracle.ve_contract(net.tensors, net.labels, net.dims, net.out_labels)
    assert np.abs(hi - ref).max() < 1e-15


# ------------------------------------------------------ cost metric

def test_worked_example_costs():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    costs = oracle.path_cost(g["labels"], g["dims"], [], g["path"])
    assert costs == g["expected_step_costs"]
    assert [sum(costs[0:3]), sum(costs[3:6]), sum(costs[6:8])] == g["expected_group_costs"]
    assert sum(costs) == g["expected_total"]
    nv = g["naive"]
    n_c = nv["gate_terms"] ** nv["n_gate_cuts"] * nv["wire_terms"] ** nv["n_wire_cuts"]
    assert n_c == nv["expected_C"]
    assert oracle.naive_pp_cost(n_c, nv["s"], nv["n_g"]) == nv["expected_cost"]
    # the naive oracle on the worked example as Eq. knitting sums it: one
    # summed index per cut over its QPD terms (the four gate cuts' 6, the
    # wire cut's 8; the h-TN above carries the wire cut as a 4 x 4 tensor
    # instead), random entries; it visits |C| terms and performs
    # |C| (s + n_g - 1) multiplications, counted by its own loop
    g1, g2, g3, g4, w = range(5)
    dims = [nv["gate_terms"]] * 4 + [nv["wire_terms"]]
    labels = [[g1, g2], [w, g1, g2], [w, g3, g4], [g3, g4], [g1], [g2], [g3], [g4], [w]]
    assert len(labels) == nv["s"] + nv["n_g"]
    rng = np.random.default_rng(5)
    ts = [rng.uniform(-1, 1, size=[dims[l] for l in ls]) for ls in labels]
    val, n_terms, n_mults = oracle.naive_contract_counted(ts, labels, dims, [])
    assert n_terms == nv["expected_C"]
    assert n_mults == nv["expected_cost"]
    hi, lo = oracle.ve_contract(ts, labels, dims, [])
    assert abs(float(val) - (float(hi) + float(lo))) <= 1e-12 * (1 + abs(float(hi)))


def test_slices_sum_to_the_network():
    """Fixing summed labels to each of their values and adding the slices
    gives the network's value (for scalars and open outputs)."""
    import itertools
    rng = np.random.default_rng(17)
    w = configs.grid_network(6, rows=2, cols=3)
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    for sliced in ([0], [0, 4], [1, 2, 6]):
        got = oracle.sliced_contract(w.tensors, w.labels, w.dims, w.out_labels, sliced)
        assert abs(float(got) - (float(hi) + float(lo))) <= 1e-15 * max(1.0, abs(float(hi)))
    m = configs.marginal_network(2, out_bits=3, n_cuts=2)
    ref = oracle.naive_contract(m.tensors, m.labels, m.dims, m.out_labels)[0]
    got = oracle.sliced_contract(m.tensors, m.labels, m.dims, m.out_labels, [0, 3])
    assert np.abs(got - ref).max() <= 1e-15
    # a single slice is a slice: fixing a label of a two-tensor product
    a, b = rng.uniform(-1, 1, (3, 4)), rng.uniform(-1, 1, (4, 5))
    got = oracle.sliced_contract([a, b], [[0, 1], [1, 2]], [3, 4, 5], [0, 2], [1])
    assert np.abs(got - a @ b).max() <= 1e-14


# ------------------------------------------ the oracle's QT evaluator

def test_instance_outputs_on_textbook_states():
    """Single-qubit eigenstates, a Bell pair and a GHZ state: expectation
    values and marginals known in closed form."""
    from workloads import circuits as c
    st = c.STATES
    for prep, (ex, ey, ez) in {"0": (0, 0, 1), "1": (0, 0, -1), "+": (1, 0, 0), "-": (-1, 0, 0),
                               "+i": (0, 1, 0), "-i": (0, -1, 0)}.items():
        for p, e in zip("XYZ", (ex, ey, ez)):
            out = sv.instance_outputs(c.Instance(1, [st[prep]], [], p))
            assert abs(out[0] - e) < 1e-15, (prep, p)
    bell = [("u", 0, c.H), ("cx", 0, 1)]
    for obs, e in (("ZZ", 1), ("XX", 1), ("YY", -1), ("ZI", 0), ("XZ", 0)):
        out = sv.instance_outputs(c.Instance(2, [st["0"], st["0"]], bell, obs))
        assert abs(out[0] - e) < 1e-15, obs
    ghz = [("u", 0, c.H), ("cx", 0, 1), ("cx", 1, 2)]
    out = sv.instance_outputs(c.Instance(3, [st["0"]] * 3, ghz, "III", kept=[0, 1, 2]))
    assert np.allclose(out, [0.5, 0, 0, 0, 0, 0, 0, 0.5], atol=1e-15)
    # kept order: x row-major over the kept list, first slowest
    out = sv.instance_outputs(c.Instance(2, [st["0"], st["1"]], [], "II", kept=[1, 0]))
    assert np.allclose(out, [0, 0, 1, 0])
    # a projection keeps the branch's weight; with Z on that qubit the sign
    proj = [("u", 0, c.H), ("proj", 0, 1)]
    assert abs(sv.instance_outputs(c.Instance(1, [st["0"]], proj, "I"))[0] - 0.5) < 1e-15
    assert abs(sv.instance_outputs(c.Instance(1, [st["0"]], proj, "Z"))[0] + 0.5) < 1e-15
    # RZZ(theta) on |++>: <X I> = cos(theta) (X I anticommutes with Z Z),
    # <X X> = 1 (it commutes)
    th = 0.7
    out = sv.instance_outputs(c.Instance(2, [st["+"], st["+"]], [("rzz", 0, 1, th)], "XI"))
    assert abs(out[0] - np.cos(th)) < 1e-15
    out = sv.instance_outputs(c.Instance(2, [st["+"], st["+"]], [("rzz", 0, 1, th)], "XX"))
    assert abs(out[0] - 1.0) < 1e-15


@pytest.mark.parametrize("seed", range(3))
def test_cut_marginal_equals_the_uncut_distribution(seed):
    """The marginal of a circuit cut by two or three wire cuts, rebuilt from
    its two QTs (Pauli-basis measurements and signed preparations), equals
    the uncut circuit's output distribution over the kept qubits."""
    from workloads import circuits as c
    for kw in ({}, {"n_left": 7, "n_right": 6, "n_cuts": 3, "kept_left": 2, "kept_right": 4}):
        cn = c.cut_marginal(seed, **kw)
        net = sv.network(cn)
        got, _ = oracle.naive_contract(net.tensors, net.labels, net.dims, net.out_labels)
        full = sv.full_value(cn)
        assert np.abs(got.reshape(-1) - full).max() < 1e-14
        assert abs(full.sum() - 1.0) < 1e-13
