"""CPU oracle for h-TN contraction — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementations that the GPU
library is checked against.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  The GPU library never imports it, and it imports nothing from the
GPU library.

Contents
  naive_contract   Eq. knitting (Sec. 2.1) written out: sum over every
                   assignment of every summed label of the product of one
                   entry per tensor (C, FP64 + Neumaier).  Generalised to
                   open output labels for marginal distributions.
  ve_contract      variable elimination, double-double (reference) or FP64
                   (timed CPU baseline) (C).
  sliced_contract  the sum over every assignment of chosen labels of the
                   network with those labels fixed (the slices a sliced
                   contraction sums).
  path_cost        the paper's postprocessing cost of a pairwise contraction
                   order: multiplications per step = product of the
                   extents of the union of both operands' labels
                   (Sec. 2.1 cost definition; Sec. 4.2 worked example).
  naive_pp_cost    |C| (s + n_g - 1), the cost of the naive knitting sum
                   (Sec. 2.1).
  mlp              FP64 forward/backward of the path cost model (see
                   oracle/mlp.py).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle/htn_oracle.c into oracle/liboracle.so (gcc, OpenMP)."""
    from .build_oracle import build as _b
    return _b(verbose=verbose)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    dpp = ctypes.POINTER(dp)
    lib.oracle_naive.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, i64p, dpp,
                                 ctypes.c_int, i32p, dp, i64p, i64p]
    lib.oracle_naive.restype = ctypes.c_int
    lib.oracle_ve.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, i64p, dpp,
                              ctypes.c_int, i32p, ctypes.c_int, dp, dp]
    lib.oracle_ve.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _marshal(tensors, labels, dims, out_labels):
    n_t = len(tensors)
    arrs = [np.ascontiguousarray(t, dtype=np.float64) for t in tensors]
    for a, ls in zip(arrs, labels):
        if a.ndim != len(ls):
            raise ValueError("tensor rank does not match its label list")
        for ax, l in enumerate(ls):
            if a.shape[ax] != dims[l]:
                raise ValueError("tensor extent does not match label dimension")
    ranks = np.array([len(l) for l in labels], dtype=np.int32)
    flat = np.array([x for ls in labels for x in ls] or [0], dtype=np.int32)
    d = np.array(dims, dtype=np.int64)
    outl = np.array(list(out_labels) or [0], dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    ptrs = (dp * n_t)(*[a.ctypes.data_as(dp) for a in arrs])
    n_o = int(np.prod([dims[l] for l in out_labels])) if out_labels else 1
    keep = (arrs, ranks, flat, d, outl, ptrs)
    return keep, n_o


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def naive_contract_counted(tensors, labels, dims, out_labels=()):
    """Naive knitting sum (Sec. 2.1, Eq. knitting); returns (result array
    shaped by out_labels, n_terms, multiplications the loop performed)."""
    lib = _load()
    (arrs, ranks, flat, d, outl, ptrs), n_o = _marshal(tensors, labels, dims, out_labels)
    out = np.zeros(n_o, dtype=np.float64)
    nterms = ctypes.c_int64(0)
    nmults = ctypes.c_int64(0)
    st = lib.oracle_naive(len(arrs), _p(ranks, ctypes.c_int32), _p(flat, ctypes.c_int32),
                          len(dims), _p(d, ctypes.c_int64), ptrs, len(out_labels),
                          _p(outl, ctypes.c_int32), _p(out, ctypes.c_double),
                          ctypes.byref(nterms), ctypes.byref(nmults))
    if st != 0:
        raise ValueError(f"oracle_naive failed with status {st}")
    shape = tuple(dims[l] for l in out_labels)
    return out.reshape(shape), int(nterms.value), int(nmults.value)


def naive_contract(tensors, labels, dims, out_labels=()):
    """Naive knitting sum; returns (result array shaped by out_labels, n_terms)."""
    out, n_terms, _ = naive_contract_counted(tensors, labels, dims, out_labels)
    return out, n_terms


def ve_contract(tensors, labels, dims, out_labels=(), mode="dd"):
    """Variable elimination.  mode "dd": returns (hi, lo) double-double
    arrays; mode "f64": returns the FP64 array."""
    lib = _load()
    (arrs, ranks, flat, d, outl, ptrs), n_o = _marshal(tensors, labels, dims, out_labels)
    hi = np.zeros(n_o, dtype=np.float64)
    lo = np.zeros(n_o, dtype=np.float64)
    st = lib.oracle_ve(len(arrs), _p(ranks, ctypes.c_int32), _p(flat, ctypes.c_int32),
                       len(dims), _p(d, ctypes.c_int64), ptrs, len(out_labels),
                       _p(outl, ctypes.c_int32), 1 if mode == "dd" else 0,
                       _p(hi, ctypes.c_double), _p(lo, ctypes.c_double))
    if st != 0:
        raise ValueError(f"oracle_ve failed with status {st}")
    shape = tuple(dims[l] for l in out_labels)
    if mode == "dd":
        return hi.reshape(shape), lo.reshape(shape)
    return hi.reshape(shape)


def sliced_contract(tensors, labels, dims, out_labels, sliced):
    """The network's value as the sum of its slices: for every assignment
    of the labels in `sliced` (none of them an output label), the network
    with those labels fixed (every tensor carrying one takes that index),
    contracted by ve_contract in double-double; the slices' hi and lo parts
    are summed with math.fsum (correctly rounded).  Returns an FP64 array."""
    import itertools
    import math
    vals = []
    for assign in itertools.product(*[range(dims[l]) for l in sliced]):
        fixed = dict(zip(sliced, assign))
        ts, ls = [], []
        for t, lab in zip(tensors, labels):
            a = np.asarray(t, dtype=np.float64)
            keep = []
            for ax in range(len(lab) - 1, -1, -1):
                if lab[ax] in fixed:
                    a = np.take(a, fixed[lab[ax]], axis=ax)
                else:
                    keep.append(lab[ax])
            ts.append(np.ascontiguousarray(a).reshape([dims[l] for l in reversed(keep)]) if keep
                      else np.array([float(a)]))
            ls.append(list(reversed(keep)) if keep else [len(dims)])
        d = list(dims) + [1]
        hi, lo = ve_contract(ts, ls, d, out_labels)
        vals.append((np.asarray(hi), np.asarray(lo)))
    shape = vals[0][0].shape
    out = np.zeros(shape)
    for idx in np.ndindex(*shape) if shape else [()]:
        out[idx] = math.fsum([float(h[idx]) for h, _ in vals] + [float(l[idx]) for _, l in vals])
    return out


def contract_net(net, mode="dd"):
    """Reference value of a workloads.Network: VE in double-double, hi part."""
    if mode == "naive":
        return naive_contract(net.tensors, net.labels, net.dims, net.out_labels)[0]
    r = ve_contract(net.tensors, net.labels, net.dims, net.out_labels, mode=mode)
    return r[0] if mode == "dd" else r


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# --------------------------------------------------------------------------
# cost model of the paper (integer bookkeeping, pure Python)
# --------------------------------------------------------------------------

def path_cost(labels, dims, out_labels, path):
    """Multiplications per pairwise step along an SSA path.

    Inputs are ids 0..n-1; step t consumes ids (i, j) and creates id n+t.
    A step's cost is the product of the extents of the union of both
    operands' labels (one multiplication per element of the joint index
    space, the paper's FLOP unit).  The step's result keeps a label iff a
    tensor outside the pair or the output still carries it.
    Returns the list of per-step costs.
    """
    live = {i: set(ls) for i, ls in enumerate(labels)}
    nxt = len(labels)
    outs = set(out_labels)
    costs = []
    for i, j in path:
        a, b = live.pop(i), live.pop(j)
        union = a | b
        c = 1
        for l in union:
            c *= dims[l]
        costs.append(c)
        others = set()
        for s in live.values():
            others |= s
        live[nxt] = {l for l in union if l in others or l in outs}
        nxt += 1
    return costs


def naive_pp_cost(n_coeff_terms: int, s: int, n_g: int) -> int:
    """|C| (s + n_g - 1): multiplications of the naive knitting sum."""
    return n_coeff_terms * (s + n_g - 1)
