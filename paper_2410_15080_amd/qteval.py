"""QT evaluation through the library (Sec. 6.2): marshalling of QT
specifications (instances and assembly terms) into htn_qt_eval_create, and
the evaluated QTs as device tensors.  Every amplitude and every entry is
computed by the library's kernels."""

from __future__ import annotations

import numpy as np

from . import htn

_KIND = {"u": htn.HTN_SV_U1, "cz": htn.HTN_SV_CZ, "cx": htn.HTN_SV_CX, "rzz": htn.HTN_SV_RZZ,
         "proj": htn.HTN_SV_PROJ}


def _op(op):
    kind = op[0]
    m = [0.0] * 8
    q1 = 0
    if kind == "u":
        u = np.asarray(op[2], dtype=np.complex128)
        m = [u[0, 0].real, u[0, 0].imag, u[0, 1].real, u[0, 1].imag, u[1, 0].real, u[1, 0].imag,
             u[1, 1].real, u[1, 1].imag]
    elif kind in ("cz", "cx"):
        q1 = op[2]
    elif kind == "rzz":
        q1 = op[2]
        m[0] = float(op[3])
    elif kind == "proj":
        q1 = op[2]
    return (_KIND[kind], op[1], q1, m)


class Evaluator:
    """All QTs of a list of specs evaluated by one run (one instance launch
    and one assembly launch); .run() returns one device tensor per spec."""

    def __init__(self, specs):
        insts, starts, terms, coefs = [], [0], [], []
        self.shapes, self.entry_off = [], []
        out_base = 0
        for spec in specs:
            bases = []
            for inst in spec.instances:
                init = np.array([[v[0].real, v[0].imag, v[1].real, v[1].imag] for v in inst.init])
                insts.append((inst.n_qubits, init, [_op(o) for o in inst.ops], inst.observable, list(inst.kept)))
                bases.append(out_base)
                out_base += inst.n_outputs
            self.entry_off.append(len(starts) - 1)
            self.shapes.append(tuple(spec.shape))
            for entry_terms in spec.terms:
                for k, x, c in entry_terms:
                    terms.append(bases[k] + x)
                    coefs.append(c)
                starts.append(len(terms))
        self.n_entries = len(starts) - 1
        self.handle = htn.htn_qt_eval_create(insts, np.array(starts), np.array(terms, dtype=np.int64),
                                             np.array(coefs, dtype=np.float64))

    def run(self, stream=None, outputs=None, device="cuda"):
        import torch
        entries = torch.empty(max(1, self.n_entries), dtype=torch.float64, device=device)
        htn.htn_qt_eval_run(self.handle, entries, outputs, stream)
        out = []
        for off, shape in zip(self.entry_off, self.shapes):
            n = int(np.prod(shape)) if shape else 1
            out.append(entries[off:off + n].view(shape))
        return out


def network_tensors(cnet, stream=None, device="cuda"):
    """Device tensors of a workloads.circuits CircuitNetwork: its QTs
    evaluated by the library, its CTs copied; and the Evaluator."""
    import torch
    specs = [t for t in cnet.tensors if hasattr(t, "instances")]
    ev = Evaluator(specs)
    qts = iter(ev.run(stream, device=device))
    ts = [next(qts) if hasattr(t, "instances") else torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(device)
          for t in cnet.tensors]
    return ts, ev
