"""Plain container for an h-TN instance (structure + values, no arithmetic)."""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    """A tensor network with hyperedge (einsum-style) label semantics.

    tensors:    dense arrays, row-major, last label fastest.
    labels:     labels[i] lists the label id of every mode of tensors[i].
    dims:       dims[l] is the extent of label l (shared by every tensor
                carrying l).
    out_labels: ordered labels of the result; empty means a scalar.
    kinds:      optional tag per tensor ("qt" quantum/subcircuit tensor,
                "ct" QPD coefficient tensor), informational only.
    """

    tensors: list
    labels: list
    dims: list
    out_labels: list = field(default_factory=list)
    kinds: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def n_tensors(self) -> int:
        return len(self.tensors)

    @property
    def n_labels(self) -> int:
        return len(self.dims)

    def validate(self) -> None:
        assert len(self.tensors) == len(self.labels)
        for t, ls in zip(self.tensors, self.labels):
            assert t.ndim == len(ls), (t.shape, ls)
            for ax, l in enumerate(ls):
                assert 0 <= l < len(self.dims)
                assert t.shape[ax] == self.dims[l], (t.shape, ls, self.dims[l])
            assert len(set(ls)) == len(ls), "repeated label inside one tensor"
        assert len(set(self.out_labels)) == len(self.out_labels)

    def astype(self, dtype) -> "Network":
        return Network([np.ascontiguousarray(t, dtype=dtype) for t in self.tensors],
                       [list(l) for l in self.labels], list(self.dims),
                       list(self.out_labels), list(self.kinds), dict(self.meta))

    def input_elements(self) -> int:
        return int(sum(t.size for t in self.tensors))
