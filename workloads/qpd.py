"""QPD coefficient tensors, as data.

These are the classical tensors (CTs) of the h-TN.  They are inputs to the
contraction, so they live with the input generators; tests check them
against the channel identities they encode.

* Pauli-basis wire cut, rho = 1/2 sum_P Tr(P rho) P: a dim-4 index over
  (I, Z, X, Y) carried by both sides, with weight 1/2 per term.  All four
  terms have equal weight, the property Sec. 4.3 relies on when it exempts
  the wire tensor from QPD sampling.
* CutQC-form wire tensor c_w (Sec. 4.1, Eq. wire-tensor): a 4x4 matrix over
  upstream measurements A = (I, Z, X, Y) (rows) and downstream preparations
  B = (|0>, |1>, |+>, |i>) (columns).
* CZ gate cut (Sec. 2.1, gate QPD; six single-qubit instances): the paper
  takes the decomposition from an external library and never prints the
  weights.  The weights below follow from writing CZ = (S (x) S) exp(i pi/4
  Z(x)Z) up to phase and expanding the ZZ rotation channel into local
  operations; the instance order is
      (S^dag, S^dag; +1/2), (S, S; +1/2), (M_Z, I; +1/2), (M_Z, Z; -1/2),
      (I, M_Z; +1/2), (Z, M_Z; -1/2)
  where M_Z is the signed Z measurement sigma -> P0 sigma P0 - P1 sigma P1.
  sum c = 1 and gamma = sum |c| = 3.
"""

import numpy as np

WIRE_PAULI = np.array([0.5, 0.5, 0.5, 0.5])

CW = 0.5 * np.array([[1.0, 1.0, 0.0, 0.0],
                     [1.0, -1.0, 0.0, 0.0],
                     [-1.0, -1.0, 2.0, 0.0],
                     [-1.0, -1.0, 0.0, 2.0]])
CW_ROWS = ("I", "Z", "X", "Y")
CW_COLS = ("0", "1", "+", "+i")

CZ_COEFFS = np.array([0.5, 0.5, 0.5, -0.5, 0.5, -0.5])
# (op on first qubit, op on second qubit) per instance.
CZ_INSTANCES = (("Sdg", "Sdg"), ("S", "S"), ("MZ", "I"), ("MZ", "Z"), ("I", "MZ"), ("Z", "MZ"))

# Downstream side of a Pauli-basis wire cut: the Pauli operator injected in
# place of the cut qubit's state, written as signed preparations.
PAULI_AS_PREPS = {
    "I": (("0", 1.0), ("1", 1.0)),
    "Z": (("0", 1.0), ("1", -1.0)),
    "X": (("+", 1.0), ("-", -1.0)),
    "Y": (("+i", 1.0), ("-i", -1.0)),
}
PAULI_ORDER = ("I", "Z", "X", "Y")


# Parametric ZZ rotation RZZ(theta) = exp(-i theta/2 Z(x)Z) cut on its two
# qubits (Sec. 2.1 gate QPD for a two-qubit rotation).  With c = cos(theta/2),
# s = sin(theta/2):  U rho U^dag = c^2 rho + s^2 ZZ rho ZZ - i c s [ZZ, rho],
# and the commutator term splits into a signed Z measurement on one qubit
# and an S or S^dag rotation on the other.  Six instances, in this order:
#   (I, I; c^2), (Z, Z; s^2), (M_Z, S; cs), (M_Z, S^dag; -cs),
#   (S, M_Z; cs), (S^dag, M_Z; -cs)
# so sum c = 1 and gamma = 1 + 2 |sin theta| (3 at theta = pi/2, where the
# rotation is CZ up to local phases).
RZZ_INSTANCES = (("I", "I"), ("Z", "Z"), ("MZ", "S"), ("MZ", "Sdg"), ("S", "MZ"), ("Sdg", "MZ"))


def rzz_coeffs(theta: float) -> np.ndarray:
    c, s = np.cos(0.5 * theta), np.sin(0.5 * theta)
    return np.array([c * c, s * s, c * s, -c * s, c * s, -c * s])


# General two-qubit gates (Sec. 2.1 gate QPD for an arbitrary two-qubit
# gate): in the KAK form U = (A1 (x) A2) exp(i (a XX + b YY + c ZZ)) (B1 (x) B2)
# the three rotations commute, and exp(i t P(x)P) = (V (x) V) RZZ(-2t) (V (x) V)^dag
# with V Z V^dag = P (V = H for X, S H for Y, I for Z).  Each rotation is cut
# with the six RZZ instances, every instance operation conjugated by V on
# its qubit: three cut indices of dimension 6 per gate (216 terms), weights
# rzz_coeffs(-2t) each, gamma = prod (1 + 2 |sin 2t|).
KAK_AXES = ("X", "Y", "Z")


def kak_coeffs(t: float) -> np.ndarray:
    """QPD weights of the rotation exp(i t P(x)P) (any Pauli P)."""
    return rzz_coeffs(-2.0 * t)
