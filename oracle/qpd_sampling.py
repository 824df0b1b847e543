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

Before sampling, the CTs that join the same tensors are fused (Sec. 4.3,
Sec. 6.1 Step 1): their tensor product becomes one CT on one fused index,
and every tensor carrying their labels has those modes merged into that one
index (``fuse_parallel``).  The fused network contracts to the same value;
sampling then draws each fused CT as a whole (``simplify``).

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


def parallel_groups(net: Network, cts):
    """The CTs of `cts` (rank-1 tensors) grouped by the set of other
    tensors that carry their label (the CTs "between the same QTs").
    Groups are ordered by their lowest CT id, CTs within a group ascending."""
    by_key = {}
    for c in sorted(cts):
        assert len(net.labels[c]) == 1
        lab = net.labels[c][0]
        key = tuple(t for t, ls in enumerate(net.labels) if t != c and lab in ls)
        by_key.setdefault(key, []).append(c)
    return sorted(by_key.values(), key=lambda g: g[0])


def fuse_parallel(net: Network, groups):
    """Fuse each group of CTs into one CT (their tensor product, index
    row-major over the group's labels in group order, first slowest) on the
    label of the group's first CT; every other tensor carrying the group's
    labels has those modes moved to where the first of them stood, in group
    order, and merged into one mode.  The other labels of a group stay in
    the label list but no tensor carries them (their extent becomes 1).
    Returns (fused network, [fused CT id per group])."""
    tensors = [np.asarray(t, dtype=np.float64) for t in net.tensors]
    labels = [list(l) for l in net.labels]
    dims = list(net.dims)
    kinds = list(net.kinds) if net.kinds else ["?"] * len(tensors)
    drop = set()
    fused_ids = []
    for g in groups:
        glabs = [net.labels[c][0] for c in g]
        f_lab = glabs[0]
        # the fused CT: outer product of the group's vectors
        prod = np.ones(1)
        for c in g:
            prod = np.multiply.outer(prod, tensors[c]).reshape(-1)
        tensors[g[0]] = prod
        f_dim = int(np.prod([dims[l] for l in glabs]))
        for c in g[1:]:
            drop.add(c)
        # every other tensor carrying the labels: merge the modes
        for t in range(len(tensors)):
            if t in g or not any(l in labels[t] for l in glabs):
                continue
            assert all(l in labels[t] for l in glabs), "a tensor carries only part of a group"
            pos = [labels[t].index(l) for l in glabs]     # the group's modes, in group order
            first = min(pos)
            before = [a for a in range(len(labels[t])) if a not in pos and a < first]
            after = [a for a in range(len(labels[t])) if a not in pos and a > first]
            x = np.transpose(tensors[t], before + pos + after)
            shape = [dims[labels[t][a]] for a in before] + [f_dim] + [dims[labels[t][a]] for a in after]
            tensors[t] = np.ascontiguousarray(x).reshape(shape)
            labels[t] = [labels[t][a] for a in before] + [f_lab] + [labels[t][a] for a in after]
        for l in glabs[1:]:
            dims[l] = 1
        dims[f_lab] = f_dim
        fused_ids.append(g[0])
    keep = [t for t in range(len(tensors)) if t not in drop]
    new_id = {t: k for k, t in enumerate(keep)}
    out = Network([tensors[t] for t in keep], [labels[t] for t in keep], dims, list(net.out_labels),
                  [kinds[t] for t in keep], dict(net.meta))
    return out, [new_id[f] for f in fused_ids]


def simplify(net: Network, cts, s_qpd: int, uniforms):
    """Sec. 4.3 in full: fuse the CTs of `cts` that join the same tensors,
    draw every fused CT s_qpd times (group k uses uniforms[k], s_qpd values)
    and truncate.  Returns (simplified network, fused network, fused CT ids,
    counts per fused CT)."""
    groups = parallel_groups(net, cts)
    fused, fids = fuse_parallel(net, groups)
    counts = [sample_counts(fused.tensors[f], s_qpd, uniforms[k]) for k, f in enumerate(fids)]
    return truncate(fused, fids, counts, s_qpd), fused, fids, counts


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
