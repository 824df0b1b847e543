"""Seeded generators for the five benchmark workloads.

Every function takes an explicit seed and returns :class:`Network` objects
(or lists of them).  Shapes follow the paper's workloads: subcircuits of at
most 15 qubits (Sec. 7.1) with 2-10 cuts (Sec. 7.2), six-term gate cuts
(Sec. 2.1) and four-dimensional wire-cut indices (Sec. 4.1).  None of the
paper's benchmark circuits are reproduced; these are synthetic stand-ins.

  grid_network        16 QTs on a 4x4 grid, each edge a wire (dim 4) or a
                      CZ gate cut (dim 6), entries U[-1,1].
  marginal_network    two QTs [4^c, 2^b] joined through c CutQC wire
                      tensors; result is a 2^b x 2^b marginal.
  ring_of_rings       8 rings x 8 QTs, 3-6 cut indices per QT.
  random_batch        many small random networks of uneven size.

The circuit workloads (subcircuit instances whose results form the QTs)
are in workloads.circuits.
"""

from __future__ import annotations

import numpy as np

from . import qpd
from .network import Network


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
