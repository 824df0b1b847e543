"""Tiny exact statevector simulator (complex128) standing in for a QPU.

It evaluates subcircuit instances into quantum-tensor entries (expectation
values), the role the paper's QT evaluator gives to QPUs or simulators
(Sec. 6.2), and it evaluates uncut circuits for reference values.  It is
deliberately minimal: single-qubit unitaries, CZ, state preparation of the
six Pauli eigenstates, a signed mid-circuit Z measurement, and
expectation values of Pauli strings.

Qubit q is axis q of a (2,)*n array.
"""

from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = S.conj().T
PAULI = {"I": I2, "Z": Z, "X": X, "Y": Y}

# Single-qubit states used as preparations for the downstream side of a
# wire cut.
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
        elif kind == "mz":
            q = op[1]
            rest = ops[k + 1:]
            v0 = run_ops(project(psi, q, 0), rest, observable)
            v1 = run_ops(project(psi, q, 1), rest, observable)
            return v0 - v1
        else:
            raise ValueError(kind)
    return expect_pauli_string(psi, observable)
