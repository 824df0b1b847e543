"""GPU parity of QPD sampling and truncation (Sec. 4.3) against the oracle.

* htn_qpd_sample: counts bit-exact and weights equal to the oracle's on the
  same uniforms (both decide the draws in FP64 with the same accumulation).
* htn_truncate_*: the gather is a copy, so bit-exact against numpy's take,
  for several dtypes, ranks, ragged sizes spanning many blocks, reordered
  and identity axes, many items per launch.
* End to end: grid h-TNs whose gate-cut CTs are sampled, truncated on the
  device and contracted by the library match the oracle's truncated network
  (double-double contraction) to 1e-10 relative.
"""

import numpy as np
import pytest

import oracle
from oracle import qpd_sampling as qs
from paper_2410_15080_amd import htn
from workloads import configs, qpd

from gpu_helpers import rel_err, to_device

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("s_qpd", [1, 2, 17, 1000, 100000])
def test_sampler_matches_oracle(s_qpd):
    rng = np.random.default_rng(s_qpd)
    for c in (qpd.CZ_COEFFS, np.array([0.0, 2.5, -0.1, 0.0, 1e-300, -3.0, 0.0]), np.array([-4.0])):
        u = rng.random(s_qpd)
        u[0] = np.nextafter(1.0, 0.0)
        counts, weights = htn.htn_qpd_sample(c, s_qpd, u)
        ref_c = qs.sample_counts(c, s_qpd, u)
        ref_w = qs.estimator_weights(c, ref_c, s_qpd)
        assert np.array_equal(counts, ref_c)
        assert np.array_equal(weights, ref_w)
        assert counts.sum() == s_qpd


def test_sampler_rejects_bad_input():
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_qpd_sample([0.0, 0.0], 3, [0.1, 0.2, 0.3])
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_qpd_sample([1.0, 2.0], 2, [0.5, 1.0])
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_qpd_sample([1.0, np.nan], 1, [0.5])


def _take(a, kept):
    for ax, k in enumerate(kept):
        if k is not None:
            a = np.take(a, k, axis=ax)
    return a


@pytest.mark.parametrize("dtype", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_truncate_batch_is_a_bit_exact_gather(dtype):
    torch = _torch()
    tdt = {htn.HTN_F64: torch.float64, htn.HTN_F32: torch.float32, htn.HTN_BF16: torch.bfloat16}[dtype]
    rng = np.random.default_rng(7)
    shapes = [(6,), (6, 4), (5, 6, 6, 4), (6, 6, 6, 6, 6, 2), (1, 3), (4, 4, 4, 4, 4, 4, 4, 4), (7, 1, 9)]
    items, srcs, dsts, refs = [], [], [], []
    for sh in shapes:
        kept = []
        for d in sh:
            r = rng.random()
            if r < 0.3:
                kept.append(None)
            else:
                k = rng.choice(d, size=int(rng.integers(1, d + 1)), replace=False)
                kept.append(np.sort(k) if r < 0.8 else k)  # some in shuffled order
        a = torch.from_numpy(rng.uniform(-1, 1, sh)).to(tdt)
        ref = _take(a.double().numpy(), kept)
        src = a.cuda()
        dst = torch.full(ref.shape, float("nan"), dtype=tdt, device="cuda")
        items.append((src, dst, sh, kept))
        srcs.append(src)
        dsts.append(dst)
        refs.append(ref)
    t = htn.htn_truncate_create(items, dtype)
    for _ in range(2):
        htn.htn_truncate_run(t)
        torch.cuda.synchronize()
        for dst, ref in zip(dsts, refs):
            assert np.array_equal(dst.double().cpu().numpy(), ref)
        for dst in dsts:
            dst.fill_(float("nan"))
    htn.htn_truncate_destroy(t)


def test_truncate_packs_many_small_items_with_large_ones():
    # sizes around the 1024-element block: single elements, runs that fill a
    # block exactly, items one element above and below it, and larger ones
    torch = _torch()
    rng = np.random.default_rng(11)
    shapes = ([(1,)] * 700 + [(32, 32), (1025,), (1023,), (2,), (1024, 1), (3, 7, 5), (2049,), (6, 6, 6, 6)]
              + [(4, 6)] * 300 + [(1000, 1, 1), (5,)])
    items, dsts, refs = [], [], []
    for sh in shapes:
        kept = [rng.choice(d, size=int(rng.integers(1, d + 1)), replace=False) if d > 1 and rng.random() < 0.7
                else None for d in sh]
        a = rng.uniform(-1, 1, sh)
        ref = _take(a, kept)
        dst = torch.full(ref.shape, float("nan"), dtype=torch.float64, device="cuda")
        items.append((torch.from_numpy(a).cuda(), dst, sh, kept))
        dsts.append(dst)
        refs.append(ref)
    t = htn.htn_truncate_create(items, htn.HTN_F64)
    htn.htn_truncate_run(t)
    torch.cuda.synchronize()
    got = torch.cat([d.reshape(-1) for d in dsts]).cpu().numpy()
    assert np.array_equal(got, np.concatenate([r.reshape(-1) for r in refs]))
    htn.htn_truncate_destroy(t)


def test_truncate_rejects_bad_items():
    torch = _torch()
    a = torch.zeros(6, 4, dtype=torch.float64, device="cuda")
    b = torch.zeros(6, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_truncate_create([(a, b, (6, 4), [[0, 6], None])], htn.HTN_F64)
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_truncate_create([(a, b, (6, 4), [[], None])], htn.HTN_F64)
    with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
        htn.htn_truncate_create([(a, b, (6, 0), [None, None])], htn.HTN_F64)


def sample_and_truncate(w, s_qpd, rng, dtype=htn.HTN_F64):
    """Sample every gate-cut CT of w on the library, truncate its QTs on the
    device; returns (device tensors, dims, per-CT counts, gate CT ids)."""
    torch = _torch()
    dev = to_device(w, dtype)
    gate = [i for i, t in enumerate(w.tensors) if w.kinds[i] == "ct" and t.size == 6]
    counts, kept_of = {}, {}
    new = list(dev)
    for c in gate:
        u = rng.random(s_qpd)
        n, wts = htn.htn_qpd_sample(w.tensors[c], s_qpd, u)
        counts[c] = n
        k = np.nonzero(n)[0]
        kept_of[w.labels[c][0]] = k
        new[c] = torch.from_numpy(wts[k]).to("cuda").to(dev[c].dtype)
    dims = list(w.dims)
    for lab, k in kept_of.items():
        dims[lab] = len(k)
    items = []
    for t, ls in enumerate(w.labels):
        if t in counts or not any(l in kept_of for l in ls):
            continue
        dst = torch.empty(tuple(dims[l] for l in ls), dtype=dev[t].dtype, device="cuda")
        items.append((dev[t], dst, tuple(w.dims[l] for l in ls), [kept_of.get(l) for l in ls]))
        new[t] = dst
    if items:
        tr = htn.htn_truncate_create(items, dtype)
        htn.htn_truncate_run(tr)
        torch.cuda.synchronize()
        htn.htn_truncate_destroy(tr)
    return new, dims, [counts[c] for c in gate], gate


@pytest.mark.parametrize("s_qpd", [1, 4, 64, 100000])
def test_sampled_grid_networks_match_oracle(s_qpd):
    torch = _torch()
    rng = np.random.default_rng(100 + s_qpd)
    nets, keep, refs = [], [], []
    for seed in range(6):
        w = configs.grid_network(seed)
        ts, dims, cnts, gate = sample_and_truncate(w, s_qpd, rng)
        ref_net = qs.truncate(w, gate, cnts, s_qpd)
        assert ref_net.dims == dims
        refs.append(oracle.contract_net(ref_net))
        net = htn.htn_create(ts, w.labels, dims, [], compute=htn.HTN_F64)
        htn.htn_set_path(net, htn.HTN_PATH_SAMPLED)
        nets.append(net)
        keep.append(ts)
    outs = [htn.new_output(n) for n in nets]
    htn.htn_contract_batch(nets, outs)
    torch.cuda.synchronize()
    for o, ref in zip(outs, refs):
        got = float(o.cpu().numpy()[0])
        assert rel_err(got, float(ref)) < 1e-10, (got, ref)
