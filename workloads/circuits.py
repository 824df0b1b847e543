"""Seeded circuit workloads as QT specifications: which subcircuit instances
run and how their results assemble into quantum tensors.

A quantum tensor (QT) entry is a signed combination of expectation values
of subcircuit instances (Sec. 2.1: one instance per QPD term; Sec. 6.2: the
QT evaluator turns them into classical tensors).  This module only
describes them; evaluating them is the QT evaluator's job (the library's
HIP statevector, or the oracle's).  Gate matrices and the six Pauli
eigenstates are data here.

Instance: n qubits in a product state (one 2-vector per qubit), a list of
ops, a Pauli observable (one of I, X, Y, Z per qubit) and optionally kept
qubits (observable I there): the instance has 2^len(kept) outputs,
    out[x] = Re <psi| O (x) |x><x|_kept |psi>,
x row-major over the kept qubits (first slowest), the other qubits summed
(marginalised).  Ops:
    ("u", q, U)         2x2 unitary on qubit q
    ("cz", a, b)        controlled-Z
    ("cx", c, t)        controlled-X (control c, target t)
    ("rzz", a, b, th)   exp(-i th/2 Z_a Z_b)
    ("proj", q, bit)    projection of qubit q onto |bit> (unnormalised)
A signed mid-circuit Z measurement (sigma -> P0 sigma P0 - P1 sigma P1, the
M_Z of the gate cuts) is written as two instances, one per projection,
whose results enter with signs +1 and -1 (``expand_mz``).

QTSpec: a tensor shape, its instances and, per entry (row-major over the
shape), a list of (instance, output, coefficient) terms.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

from . import qpd

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = S.conj().T

# the six Pauli eigenstates (preparations of the downstream side of a wire cut)
STATES = {
    "0": np.array([1, 0], dtype=np.complex128),
    "1": np.array([0, 1], dtype=np.complex128),
    "+": np.array([1, 1], dtype=np.complex128) / np.sqrt(2),
    "-": np.array([1, -1], dtype=np.complex128) / np.sqrt(2),
    "+i": np.array([1, 1j], dtype=np.complex128) / np.sqrt(2),
    "-i": np.array([1, -1j], dtype=np.complex128) / np.sqrt(2),
}


def rz(theta: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


@dataclass
class Instance:
    n_qubits: int
    init: list
    ops: list
    observable: str
    kept: list = field(default_factory=list)

    @property
    def n_outputs(self) -> int:
        return 1 << len(self.kept)


@dataclass
class QTSpec:
    shape: tuple
    instances: list
    terms: list  # per entry: [(instance, output, coefficient), ...]


@dataclass
class CircuitNetwork:
    """An h-TN whose QTs are given as specs: tensors[i] is a QTSpec for a QT
    or an array for a CT.  full_ops / full_qubits / full_observable /
    full_kept describe the uncut circuit (for reference values)."""
    tensors: list
    labels: list
    dims: list
    out_labels: list
    kinds: list
    full_ops: list
    full_qubits: int
    full_observable: str
    full_kept: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)


def expand_mz(ops):
    """Every ("mz", q) op split into its two projections: [(ops, sign)]."""
    out = [([], 1.0)]
    for op in ops:
        if op[0] == "mz":
            out = [(o + [("proj", op[1], b)], s * (1.0 if b == 0 else -1.0)) for o, s in out for b in (0, 1)]
        else:
            out = [(o + [op], s) for o, s in out]
    return out


class _Builder:
    """Collects instances (deduplicated by identity of their arguments) and
    entry terms for one QT."""

    def __init__(self, shape):
        self.shape = tuple(shape)
        self.instances = []
        self.terms = [[] for _ in range(int(np.prod(self.shape)) if self.shape else 1)]

    def add(self, entry, n, init, ops, observable, coef, kept=(), output=None):
        for branch_ops, sign in expand_mz(ops):
            self.instances.append(Instance(n, [np.asarray(v, np.complex128) for v in init], branch_ops,
                                           observable, list(kept)))
            k = len(self.instances) - 1
            if output is None:
                self.terms[entry].append((k, 0, coef * sign))
            else:
                for x in range(1 << len(kept)):
                    self.terms[output(x)].append((k, x, coef * sign))

    def spec(self):
        return QTSpec(self.shape, self.instances, self.terms)


# --------------------------------------------------------------------------
# 10-qubit circuit, two wire cuts, three subcircuits
# --------------------------------------------------------------------------

N_Q1 = 10
N_LAYERS1 = 4


def _block_c1(q: int, layer: int) -> int:
    """Subcircuit that owns qubit q during layer `layer` (cut after layer 1)."""
    if q <= 3:
        return 1
    if q == 4:
        return 1 if layer < 2 else 2
    if q in (5, 6):
        return 2
    if q == 7:
        return 2 if layer < 2 else 3
    return 3


def circuit1_gates(seed: int):
    """Gate list [(layer, op)] of the 10-qubit brick circuit.

    Layers 0..3: Rz(a) then Ry(b) on every qubit, then CZ on brick pairs
    (a, a+1), a = layer mod 2, kept only when both qubits belong to the same
    subcircuit at that layer.  Layer 4: a final Rz, Ry layer.  Angles are
    i.i.d. U[0, 2pi) in the order (layer, qubit, {z, y}).
    """
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(N_LAYERS1 + 1, N_Q1, 2))
    gates = []
    for layer in range(N_LAYERS1 + 1):
        for q in range(N_Q1):
            gates.append((layer, ("u", q, rz(ang[layer, q, 0]))))
            gates.append((layer, ("u", q, ry(ang[layer, q, 1]))))
        if layer < N_LAYERS1:
            for a in range(layer % 2, N_Q1 - 1, 2):
                if _block_c1(a, layer) == _block_c1(a + 1, layer):
                    gates.append((layer, ("cz", a, a + 1)))
    return gates


def _sub_ops(gates, block, qmap):
    ops = []
    for layer, op in gates:
        qs = [op[1]] if op[0] == "u" else [op[1], op[2]]
        if all(_block_c1(q, layer) == block for q in qs):
            if op[0] == "u":
                ops.append(("u", qmap[op[1]], op[2]))
            else:
                ops.append(("cz", qmap[op[1]], qmap[op[2]]))
    return ops


def circuit1_full_ops(seed: int):
    """Ops of the uncut 10-qubit circuit (same gates as the cut version)."""
    return [op for _, op in circuit1_gates(seed)]


def cut_wires(seed: int) -> CircuitNetwork:
    """10-qubit circuit, 2 wire cuts (q4, q7 after layer 1), 3 QTs.

    QT1[a]    = <Z^4 (x) P_a>   on S1 = {q0..q4}, q4 measured in Pauli a.
    QT2[a, b] = sum_prep sign * <Z^3 (x) P_b> on S2 = {q4', q5, q6, q7},
                q4' prepared per Pauli a, q7 measured in Pauli b.
    QT3[b]    = sum_prep sign * <Z^3> on S3 = {q7', q8, q9}.
    CTs: the Pauli-basis weights (1/2,1/2,1/2,1/2) on labels a and b.
    The target is <Z^(x)10> of the uncut circuit.
    """
    gates = circuit1_gates(seed)
    P = qpd.PAULI_ORDER
    zero = STATES["0"]
    b1 = _Builder((4,))
    ops1 = _sub_ops(gates, 1, {q: q for q in range(5)})
    for ia, pa in enumerate(P):
        b1.add(ia, 5, [zero] * 5, ops1, "ZZZZ" + pa, 1.0)
    b2 = _Builder((4, 4))
    ops2 = _sub_ops(gates, 2, {4: 0, 5: 1, 6: 2, 7: 3})
    for ia, pa in enumerate(P):
        for prep, sgn in qpd.PAULI_AS_PREPS[pa]:
            for ib, pb in enumerate(P):
                b2.add(ia * 4 + ib, 4, [STATES[prep], zero, zero, zero], ops2, "ZZZ" + pb, sgn)
    b3 = _Builder((4,))
    ops3 = _sub_ops(gates, 3, {7: 0, 8: 1, 9: 2})
    for ib, pb in enumerate(P):
        for prep, sgn in qpd.PAULI_AS_PREPS[pb]:
            b3.add(ib, 3, [STATES[prep], zero, zero], ops3, "ZZZ", sgn)
    return CircuitNetwork([b1.spec(), b2.spec(), b3.spec(), qpd.WIRE_PAULI.copy(), qpd.WIRE_PAULI.copy()],
                          [[0], [0, 1], [1], [0], [1]], [4, 4], [], ["qt", "qt", "qt", "ct", "ct"],
                          circuit1_full_ops(seed), N_Q1, "Z" * N_Q1, [],
                          {"config": "circuit_cut_wires", "seed": seed})


# --------------------------------------------------------------------------
# 4-qubit circuit with gate cuts
# --------------------------------------------------------------------------

_INST_U = {"S": S, "Sdg": SDG, "Z": Z, "I": I2}


def random_u2(rng) -> np.ndarray:
    """A random single-qubit unitary Rz Ry Rz with angles U[0, 2pi)."""
    a, b, c = rng.uniform(0.0, 2.0 * np.pi, size=3)
    return rz(a) @ ry(b) @ rz(c)


PAULI_M = {"X": X, "Y": Y, "Z": Z}
# V with V Z V^dag = P, per KAK axis
KAK_V = {"X": H, "Y": S @ H, "Z": I2}


def kak_gate(a1, a2, b1, b2, t):
    """The 4x4 unitary (A1 (x) A2) exp(i sum_k t_k P_k (x) P_k) (B1 (x) B2)
    (first qubit the slower index), P_k = X, Y, Z."""
    r = np.eye(4, dtype=np.complex128)
    for p, tk in zip(qpd.KAK_AXES, t):
        pp = np.kron(PAULI_M[p], PAULI_M[p])
        r = r @ (np.cos(tk) * np.eye(4) + 1j * np.sin(tk) * pp)
    return np.kron(a1, a2) @ r @ np.kron(b1, b2)


def cut_gates(seed: int, n_cuts: int = 1, n_layers: int = 3, gate: str = "cz") -> CircuitNetwork:
    """4-qubit circuit, halves {q0,q1} | {q2,q3}, crossing gate on (q1,q2) cut.

    Each layer: Rz, Ry on every qubit, CZ(0,1), CZ(2,3); the crossing gate
    follows layers 0..n_cuts-1 and is cut: CZ; with gate="general" a random
    two-qubit gate in KAK form (random single-qubit unitaries around
    exp(i (a XX + b YY + c ZZ)), a, b, c U[-pi/2, pi/2)), cut as three
    rotation cuts (three cut indices per gate); with gate="rzz" a ZZ rotation
    RZZ(theta) whose angle per cut is drawn U[-pi, pi) after the layer
    angles; with gate="cx" a CX (control q1, target q2): CX = (I (x) H) CZ
    (I (x) H), so its cut is the CZ cut with each target-side instance
    operation conjugated by H.  QTs: left[k_1..k_n] and right[k_1..k_n],
    <Z Z> of each half under instance k_i of every cut (M_Z as two signed
    projections).
    """
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(n_layers, 4, 2))
    thetas = rng.uniform(-np.pi, np.pi, size=n_cuts) if gate == "rzz" else None
    kak = None
    if gate == "general":
        # per cut: A1, A2, B1, B2 and the three rotation angles U[-pi/2, pi/2)
        kak = [(random_u2(rng), random_u2(rng), random_u2(rng), random_u2(rng),
                rng.uniform(-np.pi / 2, np.pi / 2, size=3)) for _ in range(n_cuts)]
    instances = qpd.RZZ_INSTANCES if gate in ("rzz", "general") else qpd.CZ_INSTANCES
    per_cut = 3 if gate == "general" else 1  # cut indices per crossing gate
    layers = []
    for layer in range(n_layers):
        ops = []
        for q in range(4):
            ops.append(("u", q, rz(ang[layer, q, 0])))
            ops.append(("u", q, ry(ang[layer, q, 1])))
        ops.append(("cz", 0, 1))
        ops.append(("cz", 2, 3))
        layers.append(ops)
    full = []
    for layer in range(n_layers):
        full += layers[layer]
        if layer < n_cuts:
            if gate == "general":
                full.append(("u2", 1, 2, kak_gate(*kak[layer])))
            else:
                full.append({"rzz": ("rzz", 1, 2, thetas[layer] if thetas is not None else 0.0),
                             "cx": ("cx", 1, 2)}.get(gate, ("cz", 1, 2)))

    def half_ops(side, insts):
        # side 0: global {0,1} -> local {0,1}, cut qubit local 1
        # side 1: global {2,3} -> local {0,1}, cut qubit local 0
        keep = (0, 1) if side == 0 else (2, 3)
        cutq = 1 if side == 0 else 0
        out = []
        for layer in range(n_layers):
            for op in layers[layer]:
                qs = [op[1]] if op[0] == "u" else [op[1], op[2]]
                if all(q in keep for q in qs):
                    if op[0] == "u":
                        out.append(("u", op[1] - keep[0], op[2]))
                    else:
                        out.append(("cz", op[1] - keep[0], op[2] - keep[0]))
            if layer < n_cuts and gate == "general":
                a1, a2, b1, b2, t = kak[layer]
                out.append(("u", cutq, b1 if side == 0 else b2))
                for k, p in enumerate(qpd.KAK_AXES):
                    v = KAK_V[p]
                    name = instances[insts[per_cut * layer + k]][side]
                    out.append(("u", cutq, v.conj().T))
                    out.append(("mz", cutq) if name == "MZ" else ("u", cutq, _INST_U[name]))
                    out.append(("u", cutq, v))
                out.append(("u", cutq, a1 if side == 0 else a2))
            elif layer < n_cuts:
                name = instances[insts[layer]][side]
                conj = gate == "cx" and side == 1  # the CX target's side
                if conj:
                    out.append(("u", cutq, H))
                if name == "MZ":
                    out.append(("mz", cutq))
                else:
                    out.append(("u", cutq, _INST_U[name]))
                if conj:
                    out.append(("u", cutq, H))
        return out

    shape = (6,) * (n_cuts * per_cut)
    zero = STATES["0"]
    left, right = _Builder(shape), _Builder(shape)
    for e, idx in enumerate(np.ndindex(*shape)):
        left.add(e, 2, [zero, zero], half_ops(0, idx), "ZZ", 1.0)
        right.add(e, 2, [zero, zero], half_ops(1, idx), "ZZ", 1.0)
    cut_labels = list(range(n_cuts * per_cut))
    if gate == "general":
        coeffs = [qpd.kak_coeffs(t) for g in kak for t in g[4]]
    elif gate == "rzz":
        coeffs = [qpd.rzz_coeffs(t) for t in thetas]
    else:
        coeffs = [qpd.CZ_COEFFS.copy()] * n_cuts
    return CircuitNetwork([left.spec(), right.spec()] + [np.array(c) for c in coeffs],
                          [cut_labels, cut_labels] + [[l] for l in cut_labels], [6] * len(cut_labels), [],
                          ["qt", "qt"] + ["ct"] * len(cut_labels), full, 4, "ZZZZ", [],
                          {"config": "circuit_cut_gates", "seed": seed, "n_cuts": n_cuts, "gate": gate})


# --------------------------------------------------------------------------
# Marginal distribution of a circuit cut by wire cuts into two halves
# --------------------------------------------------------------------------

def cut_marginal(seed: int, n_left: int = 6, n_right: int = 6, n_cuts: int = 2, n_layers: int = 4,
                 kept_left: int = 3, kept_right: int = 3) -> CircuitNetwork:
    """Two subcircuits joined by n_cuts wire cuts; the result is the joint
    output distribution of kept_left + kept_right qubits (the marginal
    reconstruction of the paper's workloads, with a real circuit behind it).

    Qubits 0..N-1, N = n_left + n_right - n_cuts.  Qubits n_left - n_cuts ..
    n_left - 1 belong to the left subcircuit for layers < n_layers // 2 and
    to the right one afterwards (cut between the two halves); the others
    stay on their side.  Each layer: Rz, Ry on every qubit (angles U[0,2pi)
    in (layer, qubit, {z, y}) order), then CZ on brick pairs inside one
    subcircuit.  Kept qubits: the first kept_left of the left side and the
    last kept_right of the right side (outputs x1, x2); every other qubit is
    marginalised.

    T1[a_1..a_c, x1] = <psi_L| (x)_i P_{a_i} (x) |x1><x1| |psi_L>: the cut
    qubits measured in the Pauli basis a (I, Z, X, Y).
    T2[b_1..b_c, x2] = sum over the signed preparations of each P_{b_i} of
    the probability of x2.  Pauli-basis wire CTs (1/2 each) on every cut.
    """
    rng = np.random.default_rng(seed)
    N = n_left + n_right - n_cuts
    half = n_layers // 2
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(n_layers, N, 2))
    cut0 = n_left - n_cuts

    def side(q, layer):
        if q < cut0:
            return 0
        if q < n_left:
            return 0 if layer < half else 1
        return 1

    gates = []
    for layer in range(n_layers):
        for q in range(N):
            gates.append((layer, ("u", q, rz(ang[layer, q, 0]))))
            gates.append((layer, ("u", q, ry(ang[layer, q, 1]))))
        for a in range(layer % 2, N - 1, 2):
            if side(a, layer) == side(a + 1, layer):
                gates.append((layer, ("cz", a, a + 1)))

    def sub(s, qmap):
        out = []
        for layer, op in gates:
            qs = [op[1]] if op[0] == "u" else [op[1], op[2]]
            if all(side(q, layer) == s for q in qs):
                out.append(("u", qmap[op[1]], op[2]) if op[0] == "u" else ("cz", qmap[op[1]], qmap[op[2]]))
        return out

    P = qpd.PAULI_ORDER
    zero = STATES["0"]
    kl = list(range(kept_left))
    kr_global = list(range(N - kept_right, N))
    lmap = {q: q for q in range(n_left)}
    rmap = {q: q - cut0 for q in range(cut0, N)}
    kr = [rmap[q] for q in kr_global]
    nx1, nx2 = 1 << kept_left, 1 << kept_right
    # left: observable P_a on the cut qubits
    bl = _Builder((4,) * n_cuts + (nx1,))
    opsl = sub(0, lmap)
    for ai, a in enumerate(np.ndindex(*(4,) * n_cuts)):
        obs = ["I"] * n_left
        for i, p in enumerate(a):
            obs[cut0 + i] = P[p]
        bl.add(None, n_left, [zero] * n_left, opsl, "".join(obs), 1.0, kept=kl,
               output=lambda x, ai=ai: ai * nx1 + x)
    # right: signed preparations of each P_b on the cut qubits
    br = _Builder((4,) * n_cuts + (nx2,))
    opsr = sub(1, rmap)
    for bi, b in enumerate(np.ndindex(*(4,) * n_cuts)):
        for combo in itertools.product(*[qpd.PAULI_AS_PREPS[P[p]] for p in b]):
            init = [STATES[prep] for prep, _ in combo] + [zero] * (n_right - n_cuts)
            sgn = float(np.prod([s for _, s in combo]))
            br.add(None, n_right, init, opsr, "I" * n_right, sgn, kept=kr, output=lambda x, bi=bi: bi * nx2 + x)
    c = n_cuts
    labels = [list(range(c)) + [c], list(range(c)) + [c + 1]] + [[i] for i in range(c)]
    tensors = [bl.spec(), br.spec()] + [qpd.WIRE_PAULI.copy() for _ in range(c)]
    return CircuitNetwork(tensors, labels, [4] * c + [nx1, nx2], [c, c + 1],
                          ["qt", "qt"] + ["ct"] * c, [op for _, op in gates], N, "I" * N, kl + kr_global,
                          {"config": "circuit_cut_marginal", "seed": seed})
