"""Seeded generators for the five benchmark workloads.

Every function takes an explicit seed and returns :class:`Network` objects
(or lists of them).  Shapes follow the paper's workloads: subcircuits of at
most 15 qubits (Sec. 7.1) with 2-10 cuts (Sec. 7.2), six-term gate cuts
(Sec. 2.1) and four-dimensional wire-cut indices (Sec. 4.1).  None of the
paper's benchmark circuits are reproduced; these are synthetic stand-ins.

  circuit_cut_wires   10-qubit brick circuit cut by 2 wire cuts into 3
                      subcircuits, QTs evaluated exactly by statevector.
  circuit_cut_gates   4-qubit circuit with 1 or 2 CZ gate cuts.
  grid_network        16 QTs on a 4x4 grid, each edge a wire (dim 4) or a
                      CZ gate cut (dim 6), entries U[-1,1].
  marginal_network    two QTs [4^c, 2^b] joined through c CutQC wire
                      tensors; result is a 2^b x 2^b marginal.
  ring_of_rings       8 rings x 8 QTs, 3-6 cut indices per QT.
  random_batch        many small random networks of uneven size.
"""

from __future__ import annotations

import numpy as np

from . import qpd
from . import statevector as sv
from .network import Network


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
            gates.append((layer, ("u", q, sv.rz(ang[layer, q, 0]))))
            gates.append((layer, ("u", q, sv.ry(ang[layer, q, 1]))))
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


def circuit_cut_wires(seed: int) -> Network:
    """Config: 10-qubit circuit, 2 wire cuts (q4, q7 after layer 1), 3 QTs.

    QT1[a]    = <Z^4 (x) P_a>   on S1 = {q0..q4}, q4 measured in Pauli a.
    QT2[a, b] = sum_prep sign * <Z^3 (x) P_b> on S2 = {q4', q5, q6, q7},
                q4' prepared per Pauli a, q7 measured in Pauli b.
    QT3[b]    = sum_prep sign * <Z^3> on S3 = {q7', q8, q9}.
    CTs: the Pauli-basis weights (1/2,1/2,1/2,1/2) on labels a and b.
    The target is <Z^(x)10> of the uncut circuit.
    """
    gates = circuit1_gates(seed)
    P = qpd.PAULI_ORDER
    # S1: global q0..q4 -> local 0..4
    ops1 = _sub_ops(gates, 1, {q: q for q in range(5)})
    qt1 = np.array([sv.run_ops(sv.zero_state(5), ops1, {0: "Z", 1: "Z", 2: "Z", 3: "Z", 4: p})
                    for p in P])
    # S2: q4 -> 0, q5 -> 1, q6 -> 2, q7 -> 3
    ops2 = _sub_ops(gates, 2, {4: 0, 5: 1, 6: 2, 7: 3})
    qt2 = np.zeros((4, 4))
    for ia, pa in enumerate(P):
        for prep, sgn in qpd.PAULI_AS_PREPS[pa]:
            init = sv.product_state([sv.STATES[prep], sv.STATES["0"], sv.STATES["0"], sv.STATES["0"]])
            for ib, pb in enumerate(P):
                qt2[ia, ib] += sgn * sv.run_ops(init, ops2, {0: "Z", 1: "Z", 2: "Z", 3: pb})
    # S3: q7 -> 0, q8 -> 1, q9 -> 2
    ops3 = _sub_ops(gates, 3, {7: 0, 8: 1, 9: 2})
    qt3 = np.zeros(4)
    for ib, pb in enumerate(P):
        for prep, sgn in qpd.PAULI_AS_PREPS[pb]:
            init = sv.product_state([sv.STATES[prep], sv.STATES["0"], sv.STATES["0"]])
            qt3[ib] += sgn * sv.run_ops(init, ops3, {0: "Z", 1: "Z", 2: "Z"})
    tensors = [qt1, qt2, qt3, qpd.WIRE_PAULI.copy(), qpd.WIRE_PAULI.copy()]
    labels = [[0], [0, 1], [1], [0], [1]]
    return Network(tensors, labels, [4, 4], [], ["qt", "qt", "qt", "ct", "ct"],
                   {"config": "circuit_cut_wires", "seed": seed})


# --------------------------------------------------------------------------
# 4-qubit circuit with CZ gate cuts
# --------------------------------------------------------------------------

_INST_U = {"S": sv.S, "Sdg": sv.SDG, "Z": sv.Z, "I": sv.I2}


def circuit_cut_gates(seed: int, n_cuts: int = 1, n_layers: int = 3, gate: str = "cz"):
    """4-qubit circuit, halves {q0,q1} | {q2,q3}, crossing gate on (q1,q2) cut.

    Returns (network, full_ops).  Each layer: Rz, Ry on every qubit, CZ(0,1),
    CZ(2,3); the crossing gate follows layers 0..n_cuts-1 and is cut: CZ,
    with gate="rzz" a ZZ rotation RZZ(theta) whose angle per cut is drawn
    U[-pi, pi) after the layer angles, or with gate="cx" a CX (control q1,
    target q2): CX = (I (x) H) CZ (I (x) H), so its cut is the CZ cut with
    each target-side instance operation conjugated by H.
    """
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(n_layers, 4, 2))
    thetas = rng.uniform(-np.pi, np.pi, size=n_cuts) if gate == "rzz" else None
    instances = qpd.RZZ_INSTANCES if gate == "rzz" else qpd.CZ_INSTANCES
    layers = []
    for layer in range(n_layers):
        ops = []
        for q in range(4):
            ops.append(("u", q, sv.rz(ang[layer, q, 0])))
            ops.append(("u", q, sv.ry(ang[layer, q, 1])))
        ops.append(("cz", 0, 1))
        ops.append(("cz", 2, 3))
        layers.append(ops)
    full = []
    for layer in range(n_layers):
        full += layers[layer]
        if layer < n_cuts:
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
            if layer < n_cuts:
                name = instances[insts[layer]][side]
                conj = gate == "cx" and side == 1  # the CX target's side
                if conj:
                    out.append(("u", cutq, sv.H))
                if name == "MZ":
                    out.append(("mz", cutq))
                else:
                    out.append(("u", cutq, _INST_U[name]))
                if conj:
                    out.append(("u", cutq, sv.H))
        return out

    shape = (6,) * n_cuts
    left = np.zeros(shape)
    right = np.zeros(shape)
    for idx in np.ndindex(*shape):
        left[idx] = sv.run_ops(sv.zero_state(2), half_ops(0, idx), {0: "Z", 1: "Z"})
        right[idx] = sv.run_ops(sv.zero_state(2), half_ops(1, idx), {0: "Z", 1: "Z"})
    cut_labels = list(range(n_cuts))
    coeffs = [qpd.rzz_coeffs(t) for t in thetas] if gate == "rzz" else [qpd.CZ_COEFFS.copy()] * n_cuts
    tensors = [left, right] + [np.array(c) for c in coeffs]
    labels = [cut_labels, cut_labels] + [[l] for l in cut_labels]
    net = Network(tensors, labels, [6] * n_cuts, [], ["qt", "qt"] + ["ct"] * n_cuts,
                  {"config": "circuit_cut_gates", "seed": seed, "n_cuts": n_cuts, "gate": gate})
    return net, full


# --------------------------------------------------------------------------
# Synthetic networks
# --------------------------------------------------------------------------

def _coeff(dim: int) -> np.ndarray:
    return qpd.WIRE_PAULI.copy() if dim == 4 else qpd.CZ_COEFFS.copy()


def _edges_to_network(n_nodes, edges, dims, rng, dtype, meta) -> Network:
    """QT per node over its incident edge labels (ascending), one CT per edge."""
    node_labels = [[] for _ in range(n_nodes)]
    for e, (u, v) in enumerate(edges):
        node_labels[u].append(e)
        node_labels[v].append(e)
    tensors, labels = [], []
    for ls in node_labels:
        shape = tuple(dims[l] for l in ls)
        tensors.append(rng.uniform(-1.0, 1.0, size=shape).astype(dtype))
        labels.append(list(ls))
    for e in range(len(edges)):
        tensors.append(_coeff(dims[e]).astype(dtype))
        labels.append([e])
    kinds = ["qt"] * n_nodes + ["ct"] * len(edges)
    return Network(tensors, labels, list(dims), [], kinds, meta)


def grid_network(seed: int, rows: int = 4, cols: int = 4, dtype=np.float64) -> Network:
    """4x4 grid of QTs; each of the 24 edges is a wire (4) or CZ gate (6) cut.

    Edge order: horizontal edges row by row, then vertical edges row by row.
    The cut type is drawn first (one uniform per edge, < 0.5 -> gate cut),
    then the QT entries U[-1,1] node by node.
    """
    rng = np.random.default_rng(seed)
    edges = []
    for r in range(rows):
        for c in range(cols - 1):
            edges.append((r * cols + c, r * cols + c + 1))
    for r in range(rows - 1):
        for c in range(cols):
            edges.append((r * cols + c, (r + 1) * cols + c))
    is_gate = rng.random(len(edges)) < 0.5
    dims = [6 if g else 4 for g in is_gate]
    return _edges_to_network(rows * cols, edges, dims, rng, dtype,
                             {"config": "grid", "seed": seed})


def marginal_network(seed: int, out_bits: int = 12, n_cuts: int = 4, dtype=np.float64) -> Network:
    """Two QTs [4]*n_cuts + [2^out_bits] joined through n_cuts c_w tensors.

    T1[a_1..a_c, x1] (upstream, Pauli measurement a_i on cut i) and
    T2[b_1..b_c, x2] (downstream, preparation b_i).  Each of the 4^c rows of
    T1 and of T2 is an Exp(1) draw normalised to sum 1 over the 2^out_bits
    outputs (a Dirichlet(1) quasi-distribution per cut term).  Labels:
    a_i = i, b_i = c + i, x1 = 2c, x2 = 2c + 1.  Output [x1, x2].
    """
    rng = np.random.default_rng(seed)
    rows = 4 ** n_cuts
    nx = 2 ** out_bits

    def dirichlet():
        e = rng.exponential(1.0, size=(rows, nx))
        return e / e.sum(axis=1, keepdims=True)

    t1 = dirichlet().reshape((4,) * n_cuts + (nx,))
    t2 = dirichlet().reshape((4,) * n_cuts + (nx,))
    c = n_cuts
    tensors = [t1.astype(dtype), t2.astype(dtype)]
    labels = [list(range(c)) + [2 * c], list(range(c, 2 * c)) + [2 * c + 1]]
    for i in range(c):
        tensors.append(qpd.CW.astype(dtype))
        labels.append([i, c + i])
    dims = [4] * (2 * c) + [nx, nx]
    return Network(tensors, labels, dims, [2 * c, 2 * c + 1],
                   ["qt", "qt"] + ["ct"] * c,
                   {"config": "marginal", "seed": seed, "out_bits": out_bits})


def ring_of_rings(seed: int, n_rings: int = 8, ring_len: int = 8, dtype=np.float64,
                  max_iter: int = 10000) -> Network:
    """8 rings of 8 QTs; node (r, i) = r*ring_len + i.

    Intra-ring edge (r,i)-(r,i+1) has multiplicity in {1,2,3}; inter-ring
    link (r,0)-(r+1,4) has multiplicity in {1,2}.  Multiplicities are then
    nudged (increment a random incident edge of a node with < 3 cut indices,
    decrement one of a node with > 6) until every QT has 3..6 cut indices.
    Each cut is dim 4 or 6 (50/50); entries U[-1,1].
    """
    rng = np.random.default_rng(seed)
    R, L = n_rings, ring_len
    links = []  # (u, v, kind, mult)
    for r in range(R):
        for i in range(L):
            links.append([r * L + i, r * L + (i + 1) % L, 3, int(rng.integers(1, 4))])
    for r in range(R):
        links.append([r * L + 0, ((r + 1) % R) * L + (4 % L), 2, int(rng.integers(1, 3))])
    n = R * L
    inc = [[] for _ in range(n)]
    for k, (u, v, _, _) in enumerate(links):
        inc[u].append(k)
        inc[v].append(k)
    for _ in range(max_iter):
        changed = False
        for node in range(n):
            d = sum(links[k][3] for k in inc[node])
            if d < 3:
                cand = [k for k in inc[node] if links[k][3] < links[k][2]]
                k = cand[int(rng.integers(len(cand)))]
                links[k][3] += 1
                changed = True
            elif d > 6:
                cand = [k for k in inc[node] if links[k][3] > 1]
                k = cand[int(rng.integers(len(cand)))]
                links[k][3] -= 1
                changed = True
        if not changed:
            break
    else:
        raise RuntimeError("ring_of_rings: degree adjustment did not converge")
    edges = []
    for u, v, _, m in links:
        edges += [(u, v)] * m
    dims = [6 if g else 4 for g in (rng.random(len(edges)) < 0.5)]
    return _edges_to_network(n, edges, dims, rng, dtype,
                             {"config": "ring_of_rings", "seed": seed})


def _structural_peak(n_nodes, edges, dims) -> float:
    """Largest intermediate (elements) of a size-greedy pairwise merge.

    A structural filter on shapes only: repeatedly merge the connected pair
    whose merged tensor (edges with exactly one endpoint inside) is
    smallest.  Used to reject oversized random instances.
    """
    groups = [{i} for i in range(n_nodes)]
    alive = list(range(n_nodes))

    def size(members):
        s = 1.0
        for e, (u, v) in enumerate(edges):
            if (u in members) != (v in members):
                s *= dims[e]
        return s

    peak = max(size(g) for g in groups)
    while len(alive) > 1:
        best = None
        for ia in range(len(alive)):
            for ib in range(ia + 1, len(alive)):
                ga, gb = groups[alive[ia]], groups[alive[ib]]
                connected = any((u in ga and v in gb) or (u in gb and v in ga) for u, v in edges)
                if not connected:
                    continue
                s = size(ga | gb)
                if best is None or s < best[0]:
                    best = (s, ia, ib)
        if best is None:
            break
        s, ia, ib = best
        a, b = alive[ia], alive[ib]
        groups[a] = groups[a] | groups[b]
        alive.pop(ib)
        peak = max(peak, s)
    return peak


def random_network(rng, dtype=np.float32, max_input=2 ** 22, max_peak=2 ** 24) -> Network:
    """One random small network: s ~ U{3..12} QTs, k ~ U{max(2,s-1)..14} cuts.

    A random spanning tree (node i >= 1 attaches to a uniform earlier node,
    after a random relabelling) plus k-(s-1) extra uniform random edges
    between distinct nodes (multi-edges allowed).  Cut dims 4/6 (50/50),
    entries U[-1,1].  Instances whose total input exceeds `max_input`
    elements or whose structural peak exceeds `max_peak` are redrawn.
    """
    while True:
        s = int(rng.integers(3, 13))
        k = int(rng.integers(max(2, s - 1), 15))
        perm = rng.permutation(s)
        edges = []
        for i in range(1, s):
            j = int(rng.integers(0, i))
            edges.append((int(perm[i]), int(perm[j])))
        for _ in range(k - (s - 1)):
            u, v = rng.choice(s, size=2, replace=False)
            edges.append((int(u), int(v)))
        dims = [6 if g else 4 for g in (rng.random(len(edges)) < 0.5)]
        deg_size = [1.0] * s
        for e, (u, v) in enumerate(edges):
            deg_size[u] *= dims[e]
            deg_size[v] *= dims[e]
        total = sum(deg_size) + sum(dims)
        if total > max_input:
            continue
        if _structural_peak(s, edges, dims) > max_peak:
            continue
        return _edges_to_network(s, edges, dims, rng, dtype, {"config": "random", "s": s, "k": k})


def random_batch(seed: int, n: int = 512, dtype=np.float32) -> list:
    """`n` independent random networks; network i uses rng(seed, i)."""
    out = []
    for i in range(n):
        net = random_network(np.random.default_rng([seed, i]), dtype=dtype)
        net.meta.update({"config": "random_batch", "seed": seed, "index": i})
        out.append(net)
    return out
