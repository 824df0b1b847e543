"""Fold chains (a large tensor contracted with small matrices one mode at a
time, run as one kernel launch) checked on the CPU: the kernel's index
arithmetic, replayed in numpy from the layout the planner emits, must keep
every source, matrix and destination access in bounds, write every
destination element exactly once, and give the chain's contraction."""

import json
import string

import numpy as np
import pytest

from paper_2410_15080_amd import htn
from workloads import configs
from workloads.network import Network


def _digits(a, ext):
    """Mixed-radix digits of the index array a (last axis fastest)."""
    out = []
    for e in reversed(ext):
        out.append(a % e)
        a = a // e
    return list(reversed(out))


def _replay(chain, x_data, mats, y_size):
    """The k_fold kernel's arithmetic for every outer index at once."""
    ext0, ext1 = chain["ext0"], chain["ext1"]
    n_outer = chain["n_outer"]
    f = np.arange(n_outer)
    fo = _digits(f, chain["o_ext"]) if chain["o_ext"] else []
    src_outer = sum((d * s for d, s in zip(fo, chain["o_src"])), np.zeros_like(f))
    dst_outer = sum((d * s for d, s in zip(fo, chain["o_dst"])), np.zeros_like(f))
    ext = list(ext0)
    D = int(np.prod(ext))
    a = np.arange(D)
    src_tile = sum(d * s for d, s in zip(_digits(a, ext), chain["s_src"]))
    off = src_outer[None, :] + src_tile[:, None]
    assert off.min() >= 0 and off.max() < x_data.size
    buf = x_data[off]                                   # [in-tile][outer]
    for ax, dout, m, mi, mo in zip(chain["fold_ax"], chain["fold_ext"], mats, chain["m_in"], chain["m_out"]):
        din = ext[ax]
        inner = int(np.prod(ext[ax + 1:]))
        Dn = D // din * dout
        an = np.arange(Dn)
        hi, rem = an // (dout * inner), an % (dout * inner)
        mid, lo = rem // inner, rem % inner
        new = np.zeros((Dn, n_outer))
        for k in range(din):
            moff = k * mi + mid * mo
            assert moff.min() >= 0 and moff.max() < m.size
            new += buf[(hi * din + k) * inner + lo] * m[moff][:, None]
        buf, ext, D = new, ext[:ax] + [dout] + ext[ax + 1:], Dn
    assert ext == list(ext1)
    a = np.arange(D)
    dst_tile = sum(d * s for d, s in zip(_digits(a, ext), chain["s_dst"]))
    doff = dst_outer[None, :] + dst_tile[:, None]
    assert doff.min() >= 0 and doff.max() < y_size
    assert np.bincount(doff.ravel(), minlength=y_size).tolist() == [1] * y_size  # each exactly once
    y = np.empty(y_size)
    y[doff.ravel()] = buf.ravel()
    return y


def _value_data(w, plan, vid):
    """An input value's data in its planned layout."""
    v = plan["values"][vid]
    base = v["base"]
    src_labels = list(w.labels[base])
    perm = [src_labels.index(l) for l in v["labels"]]
    return np.ascontiguousarray(np.transpose(np.asarray(w.tensors[base], dtype=np.float64), perm)).ravel()


def _chain_reference(w, plan, chain):
    """X contracted with the chain's matrices in order (einsum), laid out in
    the result value's labels."""
    letters = string.ascii_letters
    x = plan["values"][chain["x"]]
    labels = list(x["labels"])
    data = _value_data(w, plan, chain["x"]).reshape([w.dims[l] for l in labels])
    prev = chain["x"]
    for k in chain["steps"]:
        s = plan["steps"][k]
        m_id = s["b"] if s["a"] == prev else s["a"]
        prev = s["c"]
        m_base = plan["values"][m_id]["base"]
        ml = list(w.labels[m_base])
        (l,) = [q for q in ml if q in labels]
        (lp,) = [q for q in ml if q != l]
        out = [lp if q == l else q for q in labels]
        spec = "".join(letters[q] for q in labels) + "," + "".join(letters[q] for q in ml) + "->" + \
            "".join(letters[q] for q in out)
        data = np.einsum(spec, data, np.asarray(w.tensors[m_base], dtype=np.float64))
        labels = out
    y_labels = plan["values"][chain["y"]]["labels"]
    return np.ascontiguousarray(np.transpose(data, [labels.index(q) for q in y_labels])).ravel()


def _nets():
    rng = np.random.default_rng(4)
    yield configs.marginal_network(0, out_bits=8)
    yield configs.marginal_network(1, out_bits=12, n_cuts=3)
    # a chain of three folds: one axis folded twice (4 -> 3 -> 5, the second
    # matrix stored [new, old]), another 6 -> 2, two carried axes (one of
    # 3000, moved outside the tile); an explicit path makes it a chain
    x = rng.uniform(-1, 1, size=(4, 3000, 2, 6))
    m1 = rng.uniform(-1, 1, size=(4, 3))
    m2 = rng.uniform(-1, 1, size=(5, 3))
    m3 = rng.uniform(-1, 1, size=(6, 2))
    y = rng.uniform(-1, 1, size=(5, 2, 2))
    yield Network([x, m1, m2, m3, y], [[0, 1, 2, 3], [0, 4], [5, 4], [3, 6], [5, 6, 7]],
                  [4, 3000, 2, 6, 3, 5, 2, 2], [1, 2, 7])


PATHS = {2: [(0, 1), (5, 2), (6, 3), (7, 4)]}


@pytest.mark.parametrize("idx", range(3))
def test_fold_chain_layout_replays_to_the_contraction(idx):
    w = list(_nets())[idx]
    for compute in (htn.HTN_F64, htn.HTN_F32):
        ts = [np.asarray(t, dtype=np.float64 if compute == htn.HTN_F64 else np.float32) for t in w.tensors]
        n = htn.htn_create(ts, w.labels, w.dims, w.out_labels, compute=compute)
        htn.htn_set_option(n, htn.HTN_OPT_EXEC, htn.HTN_EXEC_STEPS)
        if idx in PATHS:
            htn.htn_set_path(n, PATHS[idx])
        plan = json.loads(htn.htn_plan_json(n))
        chains = plan["chains"]
        if idx < 2:  # every c_w fold is in a chain, one chain per QT
            assert len(chains) == 2 and sum(len(c["steps"]) for c in chains) == len(w.tensors) - 2
            # both chains fold network inputs: one group, launched together
            assert [c["lead"] for c in chains] == [0, 0]
        else:
            assert [len(c["steps"]) for c in chains] == [3]
        # the chains of a group run side by side: their results and the
        # workspace copies of their sources occupy disjoint bytes
        es = 8 if compute == htn.HTN_F64 else 4
        for lead in {c["lead"] for c in chains}:
            spans = []
            for c in chains:
                if c["lead"] != lead:
                    continue
                for key, vid in (("ws_y", c["y"]), ("ws_x", c["x"])):
                    if c[key] >= 0:
                        size = int(np.prod([w.dims[l] for l in plan["values"][vid]["labels"]]))
                        spans.append((c[key], c[key] + size * es))
            spans.sort()
            assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:])), spans
        for c in chains:
            assert plan["values"][c["x"]]["input"]
            # an unscaled input is read in place (its original tensor's
            # strides, no workspace copy); otherwise its planned copy
            base = plan["values"][c["x"]]["base"]
            assert c["x_raw"] == 1 and c["ws_x"] == -1
            x_data = np.asarray(w.tensors[base], dtype=np.float64).ravel()
            mats = [np.asarray(w.tensors[t], dtype=np.float64).ravel() for t in c["m_tensor"]]
            y_size = int(np.prod([w.dims[l] for l in plan["values"][c["y"]]["labels"]]))
            got = _replay(c, x_data, mats, y_size)
            ref = _chain_reference(w, plan, c)
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
            # the chain's steps after the first are not kernel steps of their own
            for pos, k in enumerate(c["steps"]):
                assert plan["steps"][k]["chain_pos"] == pos
