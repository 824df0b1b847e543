"""Circuit networks for the tests: the workloads.circuits specifications
with their QTs evaluated by the oracle's statevector, and the uncut
circuits' values."""

from oracle import statevector as sv
from workloads import circuits


def cut_wires(seed):
    """The 10-qubit two-wire-cut network (QTs by the oracle)."""
    return sv.network(circuits.cut_wires(seed))


def cut_wires_full(seed):
    """<Z^10> of the uncut 10-qubit circuit."""
    return float(sv.full_value(circuits.cut_wires(seed)))


def cut_gates(seed, n_cuts=1, gate="cz"):
    """(network with oracle QTs, <Z^4> of the uncut circuit)."""
    cn = circuits.cut_gates(seed, n_cuts, gate=gate)
    return sv.network(cn), float(sv.full_value(cn))
