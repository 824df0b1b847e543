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


# --------------------------------------------------------------------------
# Fusion of the CTs between the same QTs before sampling (Sec. 4.3)
# --------------------------------------------------------------------------

def test_fuse_matches_the_oracle_tensor_product():
    from workloads.network import Network
    rng = np.random.default_rng(5)
    for dims in ([6], [6, 6], [4, 6, 6], [2, 3, 5, 7]):
        cs = [rng.uniform(-1, 1, d) for d in dims]
        got = htn.htn_qpd_fuse(cs)
        net = Network([np.zeros(dims)] + cs, [list(range(len(dims)))] + [[k] for k in range(len(dims))],
                      list(dims), [])
        f, fids = qs.fuse_parallel(net, [list(range(1, len(dims) + 1))])
        assert np.array_equal(got, f.tensors[fids[0]])


def test_gather_merges_and_permutes_axes_bit_exactly():
    torch = _torch()
    rng = np.random.default_rng(2)
    items, refs = [], []
    for dims, groups, kept in (([4, 6, 3], [[1], [0, 2]], [None, [0, 5, 11]]),
                               ([6, 6, 4, 6], [[2], [3, 1], [0]], [None, [35, 0, 7], [1, 4]]),
                               ([5, 7], [[0, 1]], [None]),
                               ([3, 4, 5, 6, 2], [[4, 0], [2], [1, 3]], [[5, 1], None, list(range(0, 24, 5))])):
        src = rng.uniform(-1, 1, dims)
        # the reference: permute the axes into group order, merge each group
        x = np.transpose(src, [a for g in groups for a in g]).reshape([int(np.prod([dims[a] for a in g]))
                                                                       for g in groups])
        for o, k in enumerate(kept):
            if k is not None:
                x = np.take(x, k, axis=o)
        d_src = torch.from_numpy(src).cuda()
        dst = torch.empty(x.shape, dtype=torch.float64, device="cuda")
        items.append((d_src, dst, dims, groups, kept))
        refs.append(x)
    g = htn.htn_gather_create(items, htn.HTN_F64)
    htn.htn_truncate_run(g)
    torch.cuda.synchronize()
    for (_, dst, _, _, _), x in zip(items, refs):
        assert np.array_equal(dst.cpu().numpy(), x)


def _fused_case(w, seed, s_qpd):
    """Library and oracle simplification of one network on the same
    uniforms; returns the library's Simplified and the oracle's network."""
    from paper_2410_15080_amd import qpd as lq
    torch = _torch()
    gate = [i for i, k in enumerate(w.kinds) if k == "ct" and w.tensors[i].size == 6]
    n_groups = len(qs.parallel_groups(w, gate))
    rng = np.random.default_rng(seed)
    uniforms = [rng.random(s_qpd) for _ in range(n_groups)]
    ts = to_device(w)
    items = []
    lib = lq.simplify(ts, w.labels, w.dims, w.out_labels, gate, s_qpd, uniforms, items)
    ref, _, _, counts = qs.simplify(w, gate, s_qpd, uniforms)
    for a, b in zip(lib.counts, counts):
        assert np.array_equal(a, b)
    return lib, ref, items


@pytest.mark.parametrize("s_qpd", [1, 2, 8])
def test_fused_sampling_on_multi_bond_networks_matches_oracle(s_qpd):
    """Ring-of-rings networks (bond multiplicities 1-3) and random networks
    with multi-edges: the library fuses the CTs between the same QTs, draws
    the fused CTs, gathers every QT in one launch (bit-exact against the
    oracle's merged and truncated tensors) and contracts the simplified
    network to the oracle's value within 1e-10 relative (FP64)."""
    torch = _torch()
    cases = [configs.ring_of_rings(s) for s in range(2)]
    cases += [w for w in configs.random_batch(9, n=40, dtype=np.float64)
              if any(len(g) > 1 for g in qs.parallel_groups(
                  w, [i for i, k in enumerate(w.kinds) if k == "ct" and w.tensors[i].size == 6]))][:6]
    assert len(cases) >= 6
    simp, refs, items = [], [], []
    for k, w in enumerate(cases):
        lib, ref, its = _fused_case(w, 100 * s_qpd + k, s_qpd)
        simp.append(lib)
        refs.append(ref)
        items += its
    g = htn.htn_gather_create([it for it in items], htn.HTN_F64)
    htn.htn_truncate_run(g)
    torch.cuda.synchronize()
    for lib, ref in zip(simp, refs):
        assert lib.dims == ref.dims and lib.labels == ref.labels
        for a, b in zip(lib.tensors, ref.tensors):
            assert np.array_equal(a.cpu().numpy(), b)
        net = htn.htn_create(lib.tensors, lib.labels, lib.dims, lib.out_labels)
        out = htn.new_output(net)
        htn.htn_contract(net, out)
        torch.cuda.synchronize()
        hi, lo = oracle.ve_contract(ref.tensors, ref.labels, ref.dims, ref.out_labels)
        x = float(hi) + float(lo)
        assert abs(float(out.item()) - x) <= 1e-10 * abs(x) + 1e-300, (float(out.item()), x)


@pytest.mark.parametrize("s_qpd", [1, 4, 64])
def test_general_gate_cuts_fuse_their_three_rotations_before_sampling(s_qpd):
    """A general two-qubit gate cut is three rotation cuts between the same
    two QTs: the library fuses their CTs into one 216-entry CT, draws it
    jointly, gathers the QTs (bit-exact against the oracle) and contracts
    them to the oracle's value of the simplified network (FP64, 1e-10)."""
    torch = _torch()
    import circuit_nets
    for seed in (1, 2, 3):
        for n_cuts in (1,):
            w, _ = circuit_nets.cut_gates(seed, n_cuts, gate="general")
            gate = [i for i, k in enumerate(w.kinds) if k == "ct"]
            groups = qs.parallel_groups(w, gate)
            assert [len(g) for g in groups] == [3 * n_cuts]  # all rotations join the same two QTs
            lib, ref, items = _fused_case(w, 7 * s_qpd + seed, s_qpd)
            g = htn.htn_gather_create(items, htn.HTN_F64)
            htn.htn_truncate_run(g)
            torch.cuda.synchronize()
            for a, b in zip(lib.tensors, ref.tensors):
                assert np.array_equal(a.cpu().numpy(), b)
            net = htn.htn_create(lib.tensors, lib.labels, lib.dims, lib.out_labels)
            out = htn.new_output(net)
            htn.htn_contract(net, out)
            torch.cuda.synchronize()
            hi, lo = oracle.ve_contract(ref.tensors, ref.labels, ref.dims, ref.out_labels)
            x = float(hi) + float(lo)
            assert abs(float(out.item()) - x) <= 1e-10 * abs(x) + 1e-300
