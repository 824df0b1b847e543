"""Matrix-core GEMM steps against the oracle: ragged tiles, batch labels,
permuted operand layouts, all three input types."""

import json

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads.network import Network

from gpu_helpers import create, contract

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -8


def _gemm_net(rng, M, N, K, batch=1, permute=False):
    # labels: m=0, n=1, k=2, b=3
    dims = [M, N, K, batch]
    if permute:
        la, lb = [2, 3, 0], [1, 2, 3]      # A[k][b][m], B[n][k][b]
    else:
        la, lb = [3, 0, 2], [3, 1, 2]      # A[b][m][k], B[b][n][k]
    a = rng.uniform(-1, 1, size=[dims[l] for l in la])
    b = rng.uniform(-1, 1, size=[dims[l] for l in lb])
    return Network([a, b], [la, lb], dims, [3, 0, 1])


@pytest.mark.parametrize("shape", [(256, 256, 64, 1, False), (300, 200, 136, 1, False),
                                   (257, 129, 48, 3, True), (64, 1000, 40, 2, True)])
@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_gemm_step_matches_oracle(shape, compute):
    M, N, K, B, perm = shape
    w = _gemm_net(np.random.default_rng(M + N + K), M, N, K, B, perm)
    fs = htn.HTN_SUM_PLAIN if compute == htn.HTN_F64 else htn.HTN_SUM_FP64
    net = create(w, compute=compute, final_sum=fs, storage=htn.HTN_F64, exec_mode=htn.HTN_EXEC_STEPS)
    plan = json.loads(htn.htn_plan_json(net))
    assert plan["steps"][-1]["mfma"] == 1
    got = contract(net, (B, M, N))
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = hi + lo
    err = float(np.abs(got - ref).max())
    # |sum_k a b| error bound: gamma_K(u) * sum_k |a||b| <= gamma_K * K (entries in [-1,1])
    if compute == htn.HTN_F64:
        bound = K * 2.0 ** -52 * K
    elif compute == htn.HTN_F32:
        bound = (K + 2) * U32 * K
    else:
        bound = (2 * U16 + (K + 2) * U32) * K
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_split_k_gemm_matches_oracle(compute):
    """Few output tiles and a long K: the GEMM runs as parallel K ranges
    (ragged last range) whose partial products are summed in order."""
    M, N, K = 200, 150, 4100
    w = _gemm_net(np.random.default_rng(5), M, N, K, 1, False)
    fs = htn.HTN_SUM_PLAIN if compute == htn.HTN_F64 else htn.HTN_SUM_FP64
    net = create(w, compute=compute, final_sum=fs, storage=htn.HTN_F64, exec_mode=htn.HTN_EXEC_STEPS)
    step = json.loads(htn.htn_plan_json(net))["steps"][-1]
    assert step["mfma"] == 1 and step["ksplit"] > 1
    got = contract(net, (1, M, N))
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    err = float(np.abs(got - (hi + lo)).max())
    if compute == htn.HTN_F64:
        bound = K * 2.0 ** -52 * K
    elif compute == htn.HTN_F32:
        bound = (K + 2) * U32 * K
    else:
        bound = (2 * U16 + (K + 2) * U32) * K
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("final_sum", [htn.HTN_SUM_PLAIN, htn.HTN_SUM_COMPENSATED])
@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32])
def test_split_sum_long_reductions(final_sum, compute):
    """A scalar (and a 3-entry vector) summing 589 824 products: the
    per-step kernel splits each sum over many lane groups and combines the
    partials in a second pass."""
    rng = np.random.default_rng(9)
    for out in ([], [2]):
        dims = [768, 768, 3]
        la, lb = [0, 1, 2], [1, 0]
        a = rng.uniform(-1, 1, size=(768, 768, 3))
        b = rng.uniform(-1, 1, size=(768, 768))
        w = Network([a, b], [la, lb], dims, out)
        if not out:
            w = Network([a[..., 0], b], [[0, 1], lb], dims[:2], [])
        net = create(w, compute=compute, final_sum=final_sum, storage=htn.HTN_F64, exec_mode=htn.HTN_EXEC_STEPS)
        step = json.loads(htn.htn_plan_json(net))["steps"][-1]
        assert step["split"] > 1
        shape = tuple(w.dims[l] for l in w.out_labels)
        got = contract(net, shape)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = np.asarray(hi + lo)
        u = 2.0 ** -53 if compute == htn.HTN_F64 else U32
        # every partial is a chain of at most 32 products plus a 6-level
        # lane tree in the compute type, then FP64: |err| <= 2 * 40 u sum |a b|
        absum = oracle.ve_contract([np.abs(t) for t in w.tensors], w.labels, w.dims, w.out_labels)[0]
        bound = 80 * u * np.asarray(absum).max()
        assert float(np.abs(got - ref).max()) <= bound


@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_gemm_with_more_tiles_than_resident_workgroups(compute):
    """More output tiles than two per CU, ragged in M, N and K and batched:
    each workgroup walks several tiles and loads the next tile's first K
    slice while finishing the current one."""
    M, N, K, B = 2600, 2050, 24, 2
    w = _gemm_net(np.random.default_rng(11), M, N, K, B, False)
    fs = htn.HTN_SUM_PLAIN if compute == htn.HTN_F64 else htn.HTN_SUM_FP64
    net = create(w, compute=compute, final_sum=fs, storage=htn.HTN_F64, exec_mode=htn.HTN_EXEC_STEPS)
    step = json.loads(htn.htn_plan_json(net))["steps"][-1]
    assert step["mfma"] == 1 and step["ksplit"] == 1
    rows = 128 if compute == htn.HTN_F64 else 64  # workgroup tile rows
    assert -(-M // rows) * -(-N // 128) * B > 2 * 304  # above two per CU on any current part
    got = contract(net, (B, M, N))
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    err = float(np.abs(got - (hi + lo)).max())
    if compute == htn.HTN_F64:
        bound = K * 2.0 ** -52 * K
    elif compute == htn.HTN_F32:
        bound = (K + 2) * U32 * K
    else:
        bound = (2 * U16 + (K + 2) * U32) * K
    assert err <= bound, (err, bound)
