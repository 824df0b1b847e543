"""Helpers shared by the GPU tests: move a workloads.Network to the device,
contract it through the C ABI, compare with the oracle."""

import numpy as np

from paper_2410_15080_amd import htn

_TORCH_DT = {htn.HTN_F64: "float64", htn.HTN_F32: "float32", htn.HTN_BF16: "bfloat16"}


def to_device(w, storage=htn.HTN_F64):
    import torch
    dt = getattr(torch, _TORCH_DT[storage])
    return [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to("cuda").to(dt) for t in w.tensors]


def create(w, compute=htn.HTN_F64, final_sum=htn.HTN_SUM_PLAIN, storage=None, exec_mode=htn.HTN_EXEC_AUTO,
           path=None, lds=None, on_device=True):
    storage = compute if storage is None else storage
    if on_device:
        ts = to_device(w, storage)
    else:
        ts = [np.ascontiguousarray(t, dtype={0: np.float64, 1: np.float32}[storage]) for t in w.tensors]
    net = htn.htn_create(ts, w.labels, w.dims, w.out_labels, compute=compute, final_sum=final_sum,
                         storage=storage)
    if lds is not None:
        htn.htn_set_option(net, htn.HTN_OPT_FUSED_LDS_BYTES, lds)
    if path is not None:
        htn.htn_set_path(net, path)
    htn.htn_set_option(net, htn.HTN_OPT_EXEC, exec_mode)
    return net


def contract(net, shape):
    import torch
    out = htn.new_output(net)
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)[: int(np.prod(shape)) if shape else 1].reshape(shape)


def run(w, **kw):
    net = create(w, **kw)
    return contract(net, tuple(w.dims[l] for l in w.out_labels))


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (scale if scale > 0 else 1.0))
