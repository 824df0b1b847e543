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
