"""The batch work queue: networks run step by step inside one persistent
launch (input materialisations, step blocks, split-sum second passes,
matrix-core tiles and split-K sums as tasks with dependency counters).

The queue runs the per-step kernels' own task bodies on the same plan, so
every network must come out bit for bit equal to its per-step launches,
and equal to the oracle within the precision's bound."""

import json

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads import configs
from workloads.network import Network

from gpu_helpers import create

pytestmark = pytest.mark.gpu


def _gemm_net(rng, M, N, K, batch=1, permute=False):
    dims = [M, N, K, batch]
    la, lb = ([2, 3, 0], [1, 2, 3]) if permute else ([3, 0, 2], [3, 1, 2])
    a = rng.uniform(-1, 1, size=[dims[l] for l in la])
    b = rng.uniform(-1, 1, size=[dims[l] for l in lb])
    return Network([a, b], [la, lb], dims, [3, 0, 1])


def _split_sum_net(rng):
    a = rng.uniform(-1, 1, size=(768, 768, 3))
    b = rng.uniform(-1, 1, size=(768, 768))
    return Network([a, b], [[0, 1, 2], [1, 0]], [768, 768, 3], [2])


def _workloads(kind):
    rng = np.random.default_rng(21)
    if kind == "ring_random":
        return [configs.ring_of_rings(s) for s in range(3)] + configs.random_batch(7, n=24, dtype=np.float64)
    if kind == "gemm":  # ragged tiles, a batch label with permuted operands, split K
        return [_gemm_net(rng, 300, 200, 136), _gemm_net(rng, 257, 129, 48, 3, True),
                _gemm_net(rng, 200, 150, 4100)]
    a = rng.uniform(-1, 1, size=(768, 768))
    return [_split_sum_net(rng), Network([a, a.T.copy()], [[0, 1], [1, 0]], [768, 768], [])]


def _run_batch(nets, outs, graph=False, reps=1):
    import torch
    b = htn.htn_batch_create(nets)
    if graph:
        htn.htn_batch_set_graph(b, True)
    stream = torch.cuda.Stream()
    results = []
    for _ in range(reps):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            htn.htn_batch_run(b, htn.pointer_array(outs), stream)
        stream.synchronize()
        results.append([o.cpu().numpy().copy() for o in outs])
    return b, results


def _fs(compute):
    return htn.HTN_SUM_COMPENSATED if compute == htn.HTN_F64 else htn.HTN_SUM_FP64


@pytest.mark.parametrize("kind", ["ring_random", "gemm", "split_sum"])
@pytest.mark.parametrize("compute", [htn.HTN_F64, htn.HTN_F32, htn.HTN_BF16])
def test_queue_matches_per_step_launches_bit_for_bit(compute, kind):
    """Every network forced into the queue against the same networks run
    with one launch per step on side streams."""
    ws = _workloads(kind)
    queued = [create(w, compute=compute, final_sum=_fs(compute), storage=htn.HTN_F64) for w in ws]
    stepped = [create(w, compute=compute, final_sum=_fs(compute), storage=htn.HTN_F64,
                      exec_mode=htn.HTN_EXEC_STEPS) for w in ws]
    for n in queued:
        htn.htn_set_option(n, htn.HTN_OPT_QUEUE, 1)
    for n in stepped:
        htn.htn_set_option(n, htn.HTN_OPT_QUEUE, 2)
    if kind == "gemm":
        assert all(json.loads(htn.htn_plan_json(n))["steps"][-1]["mfma"] for n in queued)
    if kind == "split_sum":
        assert all(json.loads(htn.htn_plan_json(n))["steps"][-1]["split"] > 1 for n in queued)
    qo = [htn.new_output(n) for n in queued]
    so = [htn.new_output(n) for n in stepped]
    bq, rq = _run_batch(queued, qo)
    bs, rs = _run_batch(stepped, so)
    n_q, n_tasks, err = htn.htn_batch_queue_info(bq)
    assert err == 0
    assert htn.htn_batch_queue_info(bs)[:2] == (0, 0)
    # one matrix-core (input, output) type pair per queue: with mixed pairs
    # (FP32/BF16 rings) some networks stay on per-step launches
    assert n_q == len(ws) if (kind != "ring_random" or compute == htn.HTN_F64) else n_q >= 1
    assert n_tasks > n_q
    for i, (a, b) in enumerate(zip(rq[0], rs[0])):
        assert np.array_equal(a, b), i
    if compute == htn.HTN_F64 and kind != "gemm":
        for i, w in enumerate(ws[:3]):
            hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
            ref = np.asarray(hi) + np.asarray(lo)
            got = rq[0][i][: ref.size]
            assert np.abs(got - ref.reshape(-1)).max() <= 1e-10 * np.abs(ref).max(), i
    htn.htn_batch_destroy(bq)
    htn.htn_batch_destroy(bs)


def test_queue_graph_replays_and_stamps_config5_precision():
    """The random serving batch at FP32 with an FP64 final sum: the eight
    largest networks go to the queue, the rest to the fused launch (or, the
    rest of the large ones, to per-step launches); graph replays
    equal the eager run, every network is within the first-order FP32
    bound of the oracle, and every network has start and end stamps."""
    import torch
    ws = configs.random_batch(3, n=128, dtype=np.float64)
    nets = [create(w, compute=htn.HTN_F32, final_sum=htn.HTN_SUM_FP64, storage=htn.HTN_F64) for w in ws]
    heavy = np.argsort([-htn.htn_get_info(n).mults for n in nets])[:8]
    for i in heavy:  # the eight largest in the queue, whatever their step sizes
        htn.htn_set_option(nets[i], htn.HTN_OPT_QUEUE, 1)
    outs = [htn.new_output(n) for n in nets]
    b, eager = _run_batch(nets, outs)
    n_q, _, err = htn.htn_batch_queue_info(b)
    assert n_q >= 8 and err == 0
    htn.htn_batch_set_graph(b, True)
    stream = torch.cuda.Stream()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            htn.htn_batch_run(b, htn.pointer_array(outs), stream)
        stream.synchronize()
        x = torch.zeros(1 << 20, device="cuda")  # eager work between replays
        x.add_(1.0)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), eager[0][i]), (rep, i)
        t = htn.htn_batch_timestamps(b)
        assert (t[:, 1] > t[:, 0]).all() and (t[:, 0] >= -1).all(), rep
    assert htn.htn_batch_queue_info(b)[2] == 0
    u = 2.0 ** -24
    for i, w in enumerate(ws):
        if htn.htn_get_info(nets[i]).mults > 4e6 and i % 4:
            continue  # the oracle's time: a quarter of the largest networks
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ahi, alo = oracle.ve_contract([np.abs(t) for t in w.tensors], w.labels, w.dims, w.out_labels)
        n_in = len(w.tensors)
        bound = 4 * (n_in + max(w.dims)) * u * (float(ahi) + float(alo))
        assert abs(float(eager[0][i][0]) - (float(hi) + float(lo))) <= bound, i
    htn.htn_batch_destroy(b)


def test_phase_timing_runs_queue_nets_with_per_step_launches():
    """With per-step clocks requested the queue is bypassed; the results are
    the queue's, bit for bit."""
    ws = [configs.ring_of_rings(s) for s in range(3, 5)] + configs.random_batch(5, n=8, dtype=np.float64)
    nets = [create(w) for w in ws]
    for n in nets:
        htn.htn_set_option(n, htn.HTN_OPT_QUEUE, 1)
    outs = [htn.new_output(n) for n in nets]
    b, r0 = _run_batch(nets, outs)
    assert htn.htn_batch_queue_info(b)[0] == len(nets)
    htn.htn_batch_set_phase_timing(b, 64)
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        htn.htn_batch_run(b, htn.pointer_array(outs), stream)
    stream.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), r0[0][i]), i
    htn.htn_batch_destroy(b)


def test_changed_net_invalidates_the_batch():
    """A batch holds device addresses of its nets' inputs and plans: new
    data uploaded through a single contraction makes it refuse to run."""
    import torch
    w = configs.ring_of_rings(7)
    n = create(w)
    htn.htn_set_option(n, htn.HTN_OPT_QUEUE, 1)
    out = htn.new_output(n)
    b = htn.htn_batch_create([n])
    htn.htn_batch_run(b, htn.pointer_array([out]), torch.cuda.current_stream())
    torch.cuda.synchronize()
    fresh = [torch.from_numpy(np.asarray(t, dtype=np.float64)).cuda() for t in w.tensors]
    htn.htn_update_data(n, fresh)
    htn.htn_contract(n, htn.new_output(n))
    torch.cuda.synchronize()
    with pytest.raises(htn.HtnError):
        htn.htn_batch_run(b, htn.pointer_array([out]), torch.cuda.current_stream())
    htn.htn_batch_destroy(b)


def test_queue_takes_at_most_one_fused_eligible_network_per_xcd():
    """Networks that would join the work queue beyond one per XCD stay in
    the fused launch (each queued network has one XCD to itself); the batch
    still gives every network the value of its per-step launches."""
    ws = [configs.ring_of_rings(s) for s in range(24)]
    nets = [create(w) for w in ws]  # queue option left at auto
    outs = [htn.new_output(n) for n in nets]
    b, r = _run_batch(nets, outs)
    n_q, _, err = htn.htn_batch_queue_info(b)
    assert err == 0
    # 24 networks above the straggler bound of a 24-network batch, all
    # queue-eligible: at most one per XCD (an MI355X has eight)
    assert 1 <= n_q <= 8
    stepped = [create(w, exec_mode=htn.HTN_EXEC_STEPS) for w in ws]
    for n in stepped:
        htn.htn_set_option(n, htn.HTN_OPT_QUEUE, 2)
    so = [htn.new_output(n) for n in stepped]
    bs, rs = _run_batch(stepped, so)
    for i, w in enumerate(ws[:4]):
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        assert abs(float(r[0][i][0]) - ref) <= 1e-10 * abs(ref), i
        assert abs(float(rs[0][i][0]) - ref) <= 1e-10 * abs(ref), i
    htn.htn_batch_destroy(b)
    htn.htn_batch_destroy(bs)
