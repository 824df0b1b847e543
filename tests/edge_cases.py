"""Degenerate and boundary networks shared by the CPU replay and GPU
parity tests: a single tensor, extent-1 labels, pure outer products,
disconnected components, a three-way hyperedge, permuted outputs."""

import numpy as np

from workloads.network import Network


def edge_networks(seed=0):
    rng = np.random.default_rng(seed)
    u = lambda *s: rng.uniform(-1, 1, s)
    return {
        "single tensor to scalar": Network([u(3, 4)], [[0, 1]], [3, 4], []),
        "single tensor kept, transposed": Network([u(3, 4)], [[0, 1]], [3, 4], [1, 0]),
        "extent-1 labels": Network([u(1, 4), u(4, 1)], [[0, 1], [1, 2]], [1, 4, 1], [2, 0]),
        "outer product": Network([u(3), u(2)], [[0], [1]], [3, 2], [0, 1]),
        "disconnected components": Network([u(3), u(3), u(2), u(2)], [[0], [0], [1], [1]], [3, 2], []),
        "three-way hyperedge": Network([u(3), u(3, 2), u(3, 2)], [[0], [0, 1], [0, 1]], [3, 2], []),
        "output permutation": Network([u(2, 3, 4)], [[0, 1, 2]], [2, 3, 4], [2, 0, 1]),
        "dangling summed label": Network([u(3, 5), u(3)], [[0, 1], [0]], [3, 5], []),
    }
