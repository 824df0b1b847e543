"""Exact statevector simulator (complex128) — the oracle's QT evaluator,
TEST INFRASTRUCTURE ONLY (tests/, the smoke check and the bench's CPU
baseline leg may use it; the library never does).

It evaluates subcircuit instances into quantum-tensor entries (expectation
values and output marginals), the role the paper's QT evaluator gives to
QPUs or simulators (Sec. 6.2), and evaluates uncut circuits for reference
values.  Deliberately minimal and direct: numpy tensordot for single-qubit
gates, index masks for CZ / CX / RZZ / projections, expectation values by
applying the Pauli matrices and taking the inner product.

Qubit q is axis q of a (2,)*n array.
"""

from __future__ import annotations

import numpy as np

from workloads.circuits import I2, X, Y, Z, H, S, SDG, STATES, rz, ry  # noqa: F401  (gate data)

PAULI = {"I": I2, "Z": Z, "X": X, "Y": Y}


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def product_state(vecs) -> np.ndarray:
    psi = np.array(1.0, dtype=np.complex128)
    for v in vecs:
        psi = np.multiply.outer(psi, v)
    return psi


def apply_1q(psi: np.ndarray, u: np.ndarray, q: int) -> np.ndarray:
    out = np.tensordot(u, psi, axes=([1], [q]))
    return np.moveaxis(out, 0, q)


def apply_2q(psi: np.ndarray, u: np.ndarray, a: int, b: int) -> np.ndarray:
    """4x4 unitary u on qubits (a, b) (a the slower index of u)."""
    out = np.tensordot(np.asarray(u).reshape(2, 2, 2, 2), psi, axes=([2, 3], [a, b]))
    return np.moveaxis(out, [0, 1], [a, b])


def apply_cz(psi: np.ndarray, a: int, b: int) -> np.ndarray:
    out = psi.copy()
    idx = [slice(None)] * psi.ndim
    idx[a] = 1
    idx[b] = 1
    out[tuple(idx)] *= -1.0
    return out


def apply_cx(psi: np.ndarray, c: int, t: int) -> np.ndarray:
    """Flip qubit t on the amplitudes whose qubit c is 1."""
    out = psi.copy()
    idx = [slice(None)] * psi.ndim
    idx[c] = 1
    sub = out[tuple(idx)]
    ax = t if t < c else t - 1
    out[tuple(idx)] = np.flip(sub, axis=ax)
    return out


def apply_rzz(psi: np.ndarray, a: int, b: int, theta: float) -> np.ndarray:
    """exp(-i theta/2 Z_a Z_b): phase exp(-i theta/2) where the bits agree,
    exp(+i theta/2) where they differ."""
    idx = np.indices(psi.shape)
    parity = (idx[a] + idx[b]) % 2
    return psi * np.where(parity == 0, np.exp(-0.5j * theta), np.exp(0.5j * theta))


def project(psi: np.ndarray, q: int, bit: int) -> np.ndarray:
    """Unnormalised projection of qubit q onto |bit>."""
    out = np.zeros_like(psi)
    idx = [slice(None)] * psi.ndim
    idx[q] = bit
    out[tuple(idx)] = psi[tuple(idx)]
    return out


def expect_pauli_string(psi: np.ndarray, paulis: dict) -> float:
    """<psi| (x)_q paulis[q] |psi> (identity on qubits not listed)."""
    phi = psi
    for q, p in paulis.items():
        phi = apply_1q(phi, PAULI[p], q)
    return float(np.real(np.vdot(psi, phi)))


def run_ops(psi: np.ndarray, ops, observable: dict) -> float:
    """Run an op list and return the (signed) expectation of `observable`.

    ops items:
      ("u", q, 2x2 matrix)    unitary on qubit q
      ("cz", a, b)            controlled-Z
      ("rzz", a, b, theta)    exp(-i theta/2 Z_a Z_b)
      ("cx", c, t)            controlled-X (control c, target t)
      ("u2", a, b, 4x4)       two-qubit unitary on (a, b), a the slower index
      ("mz", q)               signed mid-circuit Z measurement: the result is
                              sum_b (-1)^b <O>_b over the two unnormalised
                              projected branches, each continued to the end.
    """
    for k, op in enumerate(ops):
        kind = op[0]
        if kind == "u":
            psi = apply_1q(psi, op[2], op[1])
        elif kind == "cz":
            psi = apply_cz(psi, op[1], op[2])
        elif kind == "rzz":
            psi = apply_rzz(psi, op[1], op[2], op[3])
        elif kind == "cx":
            psi = apply_cx(psi, op[1], op[2])
        elif kind == "u2":
            psi = apply_2q(psi, op[3], op[1], op[2])
        elif kind == "mz":
            q = op[1]
            rest = ops[k + 1:]
            v0 = run_ops(project(psi, q, 0), rest, observable)
            v1 = run_ops(project(psi, q, 1), rest, observable)
            return v0 - v1
        else:
            raise ValueError(kind)
    return expect_pauli_string(psi, observable)


def apply_proj(psi: np.ndarray, q: int, bit: int) -> np.ndarray:
    return project(psi, q, bit)


def instance_outputs(inst) -> np.ndarray:
    """out[x] = Re <psi| O (x) |x><x|_kept |psi> of one workloads.circuits
    Instance (x row-major over its kept qubits, first slowest)."""
    psi = product_state(inst.init)
    for op in inst.ops:
        kind = op[0]
        if kind == "u":
            psi = apply_1q(psi, op[2], op[1])
        elif kind == "cz":
            psi = apply_cz(psi, op[1], op[2])
        elif kind == "cx":
            psi = apply_cx(psi, op[1], op[2])
        elif kind == "rzz":
            psi = apply_rzz(psi, op[1], op[2], op[3])
        elif kind == "proj":
            psi = project(psi, op[1], op[2])
        else:
            raise ValueError(kind)
    phi = psi
    for q, p in enumerate(inst.observable):
        if p != "I":
            phi = apply_1q(phi, PAULI[p], q)
    out = np.zeros(1 << len(inst.kept))
    for x in range(out.size):
        idx = [slice(None)] * inst.n_qubits
        for k, q in enumerate(inst.kept):
            idx[q] = (x >> (len(inst.kept) - 1 - k)) & 1
        out[x] = float(np.real(np.vdot(psi[tuple(idx)], phi[tuple(idx)])))
    return out


def evaluate(spec) -> np.ndarray:
    """The QT a workloads.circuits QTSpec describes: every instance's
    outputs, then each entry's signed sum of its terms."""
    outs = [instance_outputs(inst) for inst in spec.instances]
    vals = np.array([sum(c * outs[k][x] for k, x, c in terms) for terms in spec.terms])
    return vals.reshape(spec.shape)


def network(cnet):
    """A workloads.Network of a workloads.circuits CircuitNetwork, its QTs
    evaluated here."""
    from workloads.network import Network
    tensors = [evaluate(t) if hasattr(t, "instances") else np.asarray(t, dtype=np.float64) for t in cnet.tensors]
    return Network(tensors, [list(l) for l in cnet.labels], list(cnet.dims), list(cnet.out_labels),
                   list(cnet.kinds), dict(cnet.meta))


def full_value(cnet) -> np.ndarray:
    """The uncut circuit's value: <O> (scalar) or, with kept qubits, the
    joint distribution over them (row-major, first kept qubit slowest)."""
    psi = zero_state(cnet.full_qubits)
    if not cnet.full_kept:
        return np.array(run_ops(psi, cnet.full_ops, {q: p for q, p in enumerate(cnet.full_observable)
                                                      if p != "I"}))
    for op in cnet.full_ops:
        if op[0] == "u":
            psi = apply_1q(psi, op[2], op[1])
        elif op[0] == "cz":
            psi = apply_cz(psi, op[1], op[2])
        else:
            raise ValueError(op[0])
    p = np.abs(psi) ** 2
    rest = tuple(q for q in range(cnet.full_qubits) if q not in cnet.full_kept)
    marg = p.sum(axis=rest)
    # axes of marg follow ascending qubit order; reorder to full_kept order
    order = sorted(cnet.full_kept)
    return np.transpose(marg, [order.index(q) for q in cnet.full_kept]).reshape(-1)
