"""htn_contract_noalloc (the allocation-free contraction) against
htn_contract on the per-step executor: the same kernels on a library-wide
static workspace instead of the net's own, so results must be identical;
two calls in a row, the second on a smaller network (the first call's
leftover workspace contents must not leak into it); and the oracle."""

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads import configs

from gpu_helpers import create

pytestmark = pytest.mark.gpu


def _ref(w):
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    return hi + lo


def _pair(w, compute=htn.HTN_F64, final_sum=htn.HTN_SUM_PLAIN):
    """The net set up by one htn_contract on the per-step executor, and that
    call's result."""
    import torch
    net = create(w, compute=compute, final_sum=final_sum, storage=compute, exec_mode=htn.HTN_EXEC_STEPS)
    out = htn.new_output(net)
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    return net, out.cpu().numpy().copy()


def test_noalloc_matches_contract_on_two_calls_in_a_row():
    import torch
    big = configs.marginal_network(2, out_bits=9)       # 512 x 512 marginal, split-K GEMM step
    small = configs.grid_network(5)                       # scalar grid network
    assert htn.htn_get_info(create(big)).workspace_bytes > htn.htn_get_info(create(small)).workspace_bytes
    nb, rb = _pair(big)
    ns, rs = _pair(small)
    ob, os_ = htn.new_output(nb), htn.new_output(ns)
    ob.fill_(float("nan"))
    os_.fill_(float("nan"))
    torch.cuda.synchronize()
    htn.htn_contract_noalloc(nb, ob)
    htn.htn_contract_noalloc(ns, os_)   # smaller input right after the larger one
    torch.cuda.synchronize()
    assert np.array_equal(ob.cpu().numpy(), rb)
    assert np.array_equal(os_.cpu().numpy(), rs)
    ref_b = _ref(big).reshape(-1)
    assert np.abs(ob.cpu().numpy() - ref_b).max() <= 1e-15
    ref_s = float(_ref(small))
    assert abs(float(os_.item()) - ref_s) <= 1e-10 * abs(ref_s)


def test_noalloc_mixed_precision_and_stream():
    """FP32 with a compensated FP64 final sum, enqueued on a side stream,
    on several networks in turn."""
    import torch
    st = torch.cuda.Stream()
    for seed in range(4):
        w = configs.grid_network(30 + seed)
        net, r = _pair(w, compute=htn.HTN_F32, final_sum=htn.HTN_SUM_COMPENSATED)
        out = htn.new_output(net)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        htn.htn_contract_noalloc(net, out, st)
        st.synchronize()
        assert np.array_equal(out.cpu().numpy(), r), seed


def test_noalloc_requires_set_up_and_bounds_the_workspace():
    import torch
    w = configs.grid_network(7)
    net = create(w, exec_mode=htn.HTN_EXEC_STEPS)
    out = htn.new_output(net)
    with pytest.raises(htn.HtnError) as e:
        htn.htn_contract_noalloc(net, out)   # no htn_contract yet
    assert e.value.name == "HTN_E_STATE"
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    htn.htn_set_path(net, htn.HTN_PATH_SAMPLED)  # the plan changed: set up again
    with pytest.raises(htn.HtnError) as e:
        htn.htn_contract_noalloc(net, out)
    assert e.value.name == "HTN_E_STATE"
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    ref = float(out.item())
    out.fill_(float("nan"))
    htn.htn_contract_noalloc(net, out)
    torch.cuda.synchronize()
    assert float(out.item()) == ref
