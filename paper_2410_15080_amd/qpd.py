"""QPD sampling of h-TNs through the library (Sec. 4.3; Step 1 of Sec. 6.1).

Orchestration only: the CTs to sample are grouped by the tensors they join
(host structure), each group's tensor product is formed by htn_qpd_fuse,
drawn by htn_qpd_sample, and every QT carrying a sampled index is gathered
(fused modes merged, undrawn indices dropped) by one htn_gather launch for
the whole batch.  Wire-cut CTs are left out by the caller (Sec. 4.3 exempts
them).

Uniforms: group k of a network (groups ordered by their lowest CT id) uses
uniforms[k], s_qpd values in [0, 1).
"""

from __future__ import annotations

import numpy as np

from . import htn


def parallel_groups(labels, cts):
    """The CTs of `cts` (rank-1) grouped by the set of other tensors that
    carry their label; groups ordered by lowest CT id, CTs ascending."""
    by_key = {}
    for c in sorted(cts):
        (lab,) = labels[c]
        key = tuple(t for t, ls in enumerate(labels) if t != c and lab in ls)
        by_key.setdefault(key, []).append(c)
    return sorted(by_key.values(), key=lambda g: g[0])


class Simplified:
    """One network after fusion, sampling and truncation: device tensors
    (gathered ones filled by the batch's gather launch), labels, extents,
    the ids of its fused CTs and their draw counts."""

    def __init__(self, tensors, labels, dims, out_labels, fused_ids, counts):
        self.tensors, self.labels, self.dims = tensors, labels, dims
        self.out_labels, self.fused_ids, self.counts = out_labels, fused_ids, counts


def simplify(tensors, labels, dims, out_labels, cts, s_qpd, uniforms, items, device="cuda"):
    """Plan one network's simplification; appends its gather items (src,
    dst, dims, groups, kept) to `items` and returns a Simplified whose
    gathered tensors hold data once the batch's gather has run.
    `tensors` are device tensors (torch), `cts` the CT ids to sample."""
    import torch
    groups = parallel_groups(labels, cts)
    labels = [list(l) for l in labels]
    dims = list(dims)
    new_labels = [list(l) for l in labels]
    kept_of = {}          # fused label -> kept fused indices
    members = {}          # fused label -> the group's labels, in group order
    drop, fused_ids, counts, cts_new = set(), [], [], {}
    for k, g in enumerate(groups):
        glabs = [labels[c][0] for c in g]
        coeffs = [tensors[c].detach().double().cpu().numpy() for c in g]
        fused = htn.htn_qpd_fuse(coeffs)
        n, w = htn.htn_qpd_sample(fused, s_qpd, uniforms[k])
        kept = np.nonzero(n)[0].astype(np.int32)
        kept_of[glabs[0]] = kept
        members[glabs[0]] = glabs
        cts_new[g[0]] = torch.from_numpy(np.ascontiguousarray(w[kept])).to(device=device, dtype=tensors[g[0]].dtype)
        drop.update(g[1:])
        fused_ids.append(g[0])
        counts.append(n)
    member_of = {l: f for f, ls in members.items() for l in ls}
    out_tensors = []
    for t, ls in enumerate(labels):
        if t in drop:
            continue
        if t in cts_new:
            out_tensors.append(cts_new[t])
            new_labels[t] = [ls[0]]
            continue
        touched = sorted({member_of[l] for l in ls if l in member_of})
        if not touched:
            out_tensors.append(tensors[t])
            continue
        # output axes: untouched modes in place; each group's modes merged
        # where the first of them stood, in group order
        groups_out, lab_out = [], []
        for a, l in enumerate(ls):
            if l not in member_of:
                groups_out.append([a])
                lab_out.append(l)
            elif a == min(ls.index(m) for m in members[member_of[l]]):
                f = member_of[l]
                groups_out.append([ls.index(m) for m in members[f]])
                lab_out.append(f)
        kept = [kept_of.get(l) if l in kept_of else None for l in lab_out]
        shape = [len(kept_of[l]) if l in kept_of else dims[l] for l in lab_out]
        dst = torch.empty(shape, dtype=tensors[t].dtype, device=device)
        items.append((tensors[t], dst, [dims[l] for l in ls], groups_out, kept))
        out_tensors.append(dst)
        new_labels[t] = lab_out
    for f, ls in members.items():
        for l in ls[1:]:
            dims[l] = 1
        dims[f] = len(kept_of[f])
    keep = [t for t in range(len(labels)) if t not in drop]
    new_id = {t: i for i, t in enumerate(keep)}
    return Simplified(out_tensors, [new_labels[t] for t in keep], dims, list(out_labels),
                      [new_id[f] for f in fused_ids], counts)
