"""Mixed precision against the double-double oracle, with stated bounds.

Bound used for scalar networks (first-order forward error of sums of
products): every term of the contraction passes through at most
n = sum over kernel steps of (summed extent + 1) roundings, so

    |x_hat - x| <= gamma(n, u) * X_abs,   gamma(n, u) = n u / (1 - n u),

where X_abs is the contraction of the same network with every entry
replaced by its absolute value (computed by the oracle) and u the unit
roundoff of the accumulation type (2^-24 for FP32).  BF16 adds the input
rounding: each of the q quantum tensors of a term is perturbed by at most
2^-8 relative, contributing q * 2^-8 * X_abs (coefficients are exact in
BF16).  Marginals use the same bounds entry-wise on max-abs error.
"""

import json

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads import configs

from gpu_helpers import create, contract, run

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -8


def _n_roundings(net):
    plan = json.loads(htn.htn_plan_json(net))
    return sum(s["n_sum"] + 1 for s in plan["steps"] if not s["absorbed"]) + 8


def _abs_value(w):
    hi, lo = oracle.ve_contract([np.abs(t) for t in w.tensors], w.labels, w.dims, w.out_labels)
    return hi + lo


def _gamma(n, u):
    return n * u / (1 - n * u)


@pytest.mark.parametrize("final_sum", [htn.HTN_SUM_FP64, htn.HTN_SUM_COMPENSATED, htn.HTN_SUM_PLAIN])
@pytest.mark.parametrize("exec_mode", [htn.HTN_EXEC_STEPS, htn.HTN_EXEC_FUSED])
def test_grid_f32_within_bound(final_sum, exec_mode):
    for seed in range(4):
        w = configs.grid_network(seed)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        net = create(w, compute=htn.HTN_F32, final_sum=final_sum, storage=htn.HTN_F64, exec_mode=exec_mode)
        got = float(contract(net, ()))
        # FP32 inputs: rounding each QT entry adds q * u to the bound
        bound = (_gamma(_n_roundings(net), U32) + 16 * U32) * float(_abs_value(w))
        assert abs(got - ref) <= bound, (seed, got, ref, bound)


@pytest.mark.parametrize("exec_mode", [htn.HTN_EXEC_STEPS, htn.HTN_EXEC_FUSED])
def test_grid_bf16_within_bound(exec_mode):
    for seed in range(4):
        w = configs.grid_network(seed)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        net = create(w, compute=htn.HTN_BF16, final_sum=htn.HTN_SUM_COMPENSATED, storage=htn.HTN_F64,
                     exec_mode=exec_mode)
        got = float(contract(net, ()))
        bound = (_gamma(_n_roundings(net), U32) + 16 * U16) * float(_abs_value(w))
        assert abs(got - ref) <= bound, (seed, got, ref, bound)


def _rounded_bf16(w):
    import torch
    out = []
    for t, kind in zip(w.tensors, w.kinds):
        x = torch.from_numpy(np.ascontiguousarray(t)).to(torch.float32).to(torch.bfloat16)
        out.append(x.to(torch.float64).numpy())
    return out


@pytest.mark.parametrize("bits", [8, 9])
@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_marginal_matrix_core_paths(compute, bits):
    """256 x 256 and 512 x 512 marginals, K = 256: the last step runs on the
    matrix cores; at 512 x 512 (above the fused kernel's batch limit) the
    folds write the GEMM operands in packed order (BF16: rounded by the
    fold) and no pack runs."""
    w = configs.marginal_network(5, out_bits=bits)
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = hi + lo
    fs = htn.HTN_SUM_PLAIN if compute == htn.HTN_F64 else htn.HTN_SUM_FP64
    net = create(w, compute=compute, final_sum=fs, storage=htn.HTN_F64, exec_mode=htn.HTN_EXEC_STEPS)
    plan = json.loads(htn.htn_plan_json(net))
    assert plan["steps"][-1]["mfma"] == 1
    assert plan["steps"][-1]["pack_id"] == ([1, 1] if bits == 9 else [0, 0])
    side = 1 << bits
    got = contract(net, (side, side))
    err = float(np.abs(got - ref).max())
    absval = _abs_value(w)
    if compute == htn.HTN_F64:
        assert err <= 1e-15
    elif compute == htn.HTN_F32:
        assert err <= float((_gamma(300, U32) + 2 * U32) * absval.max()), err
    else:
        # input rounding of the two QTs, and of the folded operand entering
        # the BF16 matrix product, plus FP32 accumulation
        rin = oracle.ve_contract(_rounded_bf16(w), w.labels, w.dims, w.out_labels, mode="f64")
        e_in = float(np.abs(rin - ref).max())
        assert err <= float((_gamma(300, U32) + 4 * U16) * absval.max()), err
        print(f"bf16 marginal: gpu max-abs {err:.3e}, input-rounding-only {e_in:.3e}")
        # sanity check only: BF16 rounding of the folded operand moves the
        # sum (its first-order bound, 3 * 2^-9 * (sum |c_w|)^4, is vacuous)
        assert abs(got.sum() - 1.0) <= 1e-2
    if compute != htn.HTN_BF16:
        assert abs(got.sum() - 1.0) <= 1e-6


def test_ring_of_rings_precisions():
    w = configs.ring_of_rings(1)
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = float(hi) + float(lo)
    absval = float(_abs_value(w))
    for compute, u_in in ((htn.HTN_F64, 0.0), (htn.HTN_F32, U32), (htn.HTN_BF16, U16)):
        net = create(w, compute=compute, final_sum=htn.HTN_SUM_COMPENSATED, storage=htn.HTN_F64)
        got = float(contract(net, ()))
        u = 2.0 ** -53 if compute == htn.HTN_F64 else U32
        bound = (_gamma(_n_roundings(net), u) + 64 * u_in) * absval
        assert abs(got - ref) <= bound, (compute, got, ref, bound)
