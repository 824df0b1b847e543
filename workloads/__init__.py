"""Seeded synthetic inputs for hybrid-tensor-network (h-TN) contraction.

This package only *produces* inputs: tensor values, integer index labels,
label dimensions and output labels, all drawn from ``numpy.random.default_rng``
with an explicit seed.  It performs none of the contraction arithmetic, so
both the CPU oracle and the GPU library can consume the same inputs without
sharing any code path that computes a result.

A network is a :class:`workloads.network.Network`: a list of dense row-major
tensors (last label fastest), one label list per tensor, a dimension per
label, and an ordered list of output labels (empty for a scalar result).
"""

from .network import Network  # noqa: F401
