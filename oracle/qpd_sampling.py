"""QPD sampling on the h-TN (Sec. 4.3) — oracle, TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may
import this module; it shares nothing with the GPU library.

Sec. 4.3 (and Step 1 of Sec. 6.1): instead of sampling global circuit
instances, the runtime samples each coefficient tensor (CT) c_x on its own:
s_QPD draws of an index i with probability |c_i| / gamma, gamma = sum_i |c_i|.
The count n_i of each index fixes how many shots its instance gets; an index
drawn zero times is dropped from the CT and from the index of every QT that
carries it (the truncation of Fig. 3 (d)).  The CT then holds the usual
unbiased QPD estimator weight per kept index, n_i * gamma * sign(c_i) / s_QPD,
whose expectation over the multinomial draw is c_i.  Wire-cut tensors are
not sampled (their terms all weigh the same).

Reading where the text is silent: a draw maps a uniform u in [0, 1) to the
first index i with u < F_i, F_i = (|c_0| + ... + |c_i|) / gamma accumulated
left to right in FP64 (inverse CDF); the uniforms are inputs, so the GPU
library and this oracle make the same draws.  A draw that lands beyond the
last non-zero weight (u >= F_last through rounding) goes to the last index
with |c_i| > 0.
"""

from __future__ import annotations

import numpy as np

from workloads.network import Network


def sample_counts(coeffs, s_qpd: int, uniforms) -> np.ndarray:
    """n_i: how many of the s_qpd draws land on index i (inverse CDF)."""
    c = np.asarray(coeffs, dtype=np.float64)
    u = np.asarray(uniforms, dtype=np.float64)
    assert u.shape == (s_qpd,)
    gamma = 0.0
    for x in c:
        gamma += abs(x)
    cdf = []
    acc = 0.0
    for x in c:
        acc += abs(x)
        cdf.append(acc / gamma)
    last = max(i for i in range(len(c)) if c[i] != 0.0)
    counts = np.zeros(len(c), dtype=np.int64)
    for x in u:
        i = 0
        while i < len(c) and not (x < cdf[i]):
            i += 1
        counts[min(i, last)] += 1
    return counts


def estimator_weights(coeffs, counts, s_qpd: int) -> np.ndarray:
    """n_i * gamma * sign(c_i) / s_qpd per index (0 where n_i = 0)."""
    c = np.asarray(coeffs, dtype=np.float64)
    gamma = 0.0
    for x in c:
        gamma += abs(x)
    return np.array([counts[i] * gamma * np.sign(c[i]) / s_qpd for i in range(len(c))])


def truncate(net: Network, sampled_cts, counts_per_ct, s_qpd: int) -> Network:
    """The simplified h-TN of Fig. 3 (d).

    sampled_cts: ids of rank-1 CTs to sample (the caller leaves wire CTs
    out); counts_per_ct[k]: the counts drawn for sampled_cts[k].  Each
    sampled CT becomes its kept indices' estimator weights, and every other
    tensor carrying its label keeps only those slices (np.take)."""
    tensors = [np.asarray(t, dtype=np.float64) for t in net.tensors]
    dims = list(net.dims)
    for ct, counts in zip(sampled_cts, counts_per_ct):
        assert len(net.labels[ct]) == 1
        lab = net.labels[ct][0]
        assert lab not in net.out_labels
        kept = [i for i in range(dims[lab]) if counts[i] > 0]
        w = estimator_weights(tensors[ct], counts, s_qpd)
        tensors[ct] = w[kept]
        for t, ls in enumerate(net.labels):
            if t != ct and lab in ls:
                tensors[t] = np.take(tensors[t], kept, axis=ls.index(lab))
        dims[lab] = len(kept)
    return Network(tensors, [list(l) for l in net.labels], dims, list(net.out_labels),
                   list(net.kinds), dict(net.meta))
