"""GPU QT evaluator (Sec. 6.2) against the oracle's statevector.

* Instance outputs: random circuits with every op kind (single-qubit
  unitaries, CZ, CX, RZZ, projections), 1 to 16 qubits (states in LDS up to
  12 qubits, in device memory above), Pauli observables with X/Y/Z mixes,
  0 to n kept qubits (both reduction shapes), against the oracle's
  instance_outputs within 1e-12.
* Assembled QTs of every circuit workload (wire cuts, CZ / RZZ / CX gate
  cuts with signed projection branches, the cut marginal) against the
  oracle's evaluate within 1e-12.
* End to end on the GPU (QTs by the evaluator, contraction by the library)
  against the uncut circuit: <Z^10>, <Z^4>, and the marginal distribution.
"""

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2410_15080_amd import htn, qteval
from workloads import circuits as c

pytestmark = pytest.mark.gpu


def _random_instance(rng, n, n_kept, n_ops=40):
    ops = []
    for _ in range(n_ops):
        kind = rng.choice(["u", "u", "cz", "cx", "rzz", "proj"] if n > 1 else ["u", "u", "proj"])
        if kind == "u":
            u = c.rz(rng.uniform(0, 2 * np.pi)) @ c.ry(rng.uniform(0, 2 * np.pi)) @ c.rz(rng.uniform(0, 2 * np.pi))
            ops.append(("u", int(rng.integers(n)), u))
        elif kind == "proj":
            if rng.random() < 0.3:  # projections sparingly: they shrink the norm
                ops.append(("proj", int(rng.integers(n)), int(rng.integers(2))))
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            ops.append((kind, a, b, rng.uniform(-np.pi, np.pi)) if kind == "rzz" else (kind, a, b))
    kept = [int(x) for x in rng.choice(n, size=n_kept, replace=False)]
    obs = [rng.choice(list("IXYZ")) for _ in range(n)]
    for q in kept:
        obs[q] = "I"
    init = []
    for _ in range(n):
        v = rng.normal(size=2) + 1j * rng.normal(size=2)
        init.append(v / np.linalg.norm(v))
    return c.Instance(n, init, ops, "".join(obs), kept)


def _spec_of(instances):
    """One entry per instance output (coefficient 1)."""
    terms = [[(k, x, 1.0)] for k, inst in enumerate(instances) for x in range(inst.n_outputs)]
    return c.QTSpec((len(terms),), instances, terms)


@pytest.mark.parametrize("sizes", [(1, 2, 3, 5, 8), (11, 12, 13), (14, 16)])
def test_instance_outputs_match_oracle(sizes):
    import torch
    rng = np.random.default_rng(sum(sizes))
    insts = []
    for n in sizes:
        for n_kept in sorted({0, 1, min(3, n), n}):
            insts.append(_random_instance(rng, n, n_kept))
    ev = qteval.Evaluator([_spec_of(insts)])
    (got,) = ev.run()
    outs = torch.empty(got.numel(), dtype=torch.float64, device="cuda")
    ev.run(outputs=outs)
    torch.cuda.synchronize()
    ref = np.concatenate([sv.instance_outputs(i) for i in insts])
    assert np.abs(got.cpu().numpy() - ref).max() <= 1e-12
    assert np.array_equal(outs.cpu().numpy(), got.cpu().numpy())


def _workloads():
    ws = [c.cut_wires(s) for s in range(2)]
    ws += [c.cut_gates(s, k, gate=g) for s in (1, 2) for k in (1, 2) for g in ("cz", "rzz", "cx")]
    ws += [c.cut_gates(s, 1, gate="general") for s in (1, 2, 3)]
    ws += [c.cut_marginal(0), c.cut_marginal(1, n_left=7, n_right=6, n_cuts=3, kept_left=2, kept_right=4)]
    return ws


def test_assembled_qts_match_oracle():
    import torch
    for cn in _workloads():
        specs = [t for t in cn.tensors if hasattr(t, "instances")]
        got = qteval.Evaluator(specs).run()
        torch.cuda.synchronize()
        for g, spec in zip(got, specs):
            ref = sv.evaluate(spec)
            assert g.shape == ref.shape
            assert np.abs(g.cpu().numpy() - ref).max() <= 1e-12, cn.meta


@pytest.mark.parametrize("exec_mode", [htn.HTN_EXEC_STEPS, htn.HTN_EXEC_FUSED])
def test_end_to_end_on_the_gpu_equals_the_uncut_circuit(exec_mode):
    import torch
    for cn in _workloads():
        ts, _ = qteval.network_tensors(cn)
        net = htn.htn_create(ts, cn.labels, cn.dims, cn.out_labels)
        htn.htn_set_option(net, htn.HTN_OPT_EXEC, exec_mode)
        out = htn.new_output(net)
        htn.htn_contract(net, out)
        torch.cuda.synchronize()
        full = sv.full_value(cn).reshape(-1)
        got = out.cpu().numpy()[: full.size]
        assert np.abs(got - full).max() <= 1e-13, cn.meta
