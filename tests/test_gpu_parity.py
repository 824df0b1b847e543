"""GPU parity: libhtn (through the C ABI) against the CPU oracle.

FP64 results must match the oracle's double-double value to 1e-10
relative (scalars) or the stated absolute bound (marginals).
"""

import random

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads import configs
import circuit_nets

from gpu_helpers import create, contract, rel_err, run

pytestmark = pytest.mark.gpu

EXECS = [htn.HTN_EXEC_STEPS, htn.HTN_EXEC_FUSED]
REL_F64 = 1e-10


@pytest.mark.parametrize("exec_mode", EXECS)
def test_wire_cut_circuit_matches_oracle_and_statevector(exec_mode):
    for seed in range(3):
        w = circuit_nets.cut_wires(seed)
        got = float(run(w, exec_mode=exec_mode))
        ref, _ = oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
        full = circuit_nets.cut_wires_full(seed)
        assert abs(got - float(ref)) <= REL_F64 * abs(float(ref))
        assert abs(got - full) < 1e-14


@pytest.mark.parametrize("gate", ["cz", "rzz", "cx", "general"])
@pytest.mark.parametrize("exec_mode", EXECS)
def test_gate_cut_circuits(exec_mode, gate):
    # CZ, parametric RZZ(theta), CX and general (KAK) two-qubit gate cuts:
    # oracle and uncut statevector
    for seed in (1, 2):
        for n_cuts in ((1,) if gate == "general" else (1, 2)):
            w, full = circuit_nets.cut_gates(seed, n_cuts, gate=gate)
            got = float(run(w, exec_mode=exec_mode))
            ref, _ = oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
            assert abs(got - float(ref)) <= 1e-13
            assert abs(got - full) <= 1e-13


@pytest.mark.parametrize("exec_mode", EXECS)
@pytest.mark.parametrize("seed", range(6))
def test_grid_f64(exec_mode, seed):
    w = configs.grid_network(seed)
    got = float(run(w, exec_mode=exec_mode))
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = float(hi) + float(lo)
    assert abs(got - ref) <= REL_F64 * abs(ref), (got, ref)


def test_grid_fused_all_in_lds_and_spilled_agree():
    """The same network with a large and a tiny LDS budget (everything
    spilled to global scratch)."""
    w = configs.grid_network(2)
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = float(hi) + float(lo)
    for lds in (163840, 65536, 32768, 24576):
        got = float(run(w, exec_mode=htn.HTN_EXEC_FUSED, lds=lds))
        assert abs(got - ref) <= REL_F64 * abs(ref), (lds, got, ref)


def _random_network(rng):
    n_labels = int(rng.integers(3, 8))
    dims = [int(d) for d in rng.integers(1, 6, size=n_labels)]
    n_t = int(rng.integers(1, 6))
    labels = []
    for _ in range(n_t):
        r = int(rng.integers(1, min(4, n_labels) + 1))
        labels.append([int(x) for x in rng.choice(n_labels, size=r, replace=False)])
    used = sorted({l for ls in labels for l in ls})
    n_out = int(rng.integers(0, 4))
    out = [int(x) for x in rng.choice(used, size=min(n_out, len(used)), replace=False)]
    tensors = [rng.uniform(-1, 1, size=[dims[l] for l in ls]) for ls in labels]
    from workloads.network import Network
    return Network(tensors, labels, dims, out)


@pytest.mark.parametrize("exec_mode", EXECS)
def test_random_networks_hyperedges_outputs_dangling_labels(exec_mode):
    """Arbitrary label layouts: hyperedges in 3+ tensors, labels summed out
    of one tensor, open outputs in any order, size-1 extents, one tensor."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        w = _random_network(rng)
        got = run(w, exec_mode=exec_mode)
        ref, _ = oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def _random_connected_path(labels, rng, dims=None, k=4):
    """A random order of pairwise steps between tensors that share a label.
    With `dims`, each step is drawn among the k sharing pairs of fewest
    multiplications (random orders that stay near the cheap ones, so their
    intermediates stay small)."""
    live = {i: set(ls) for i, ls in enumerate(labels)}
    nxt = len(labels)
    path = []
    while len(live) > 1:
        ids = sorted(live)
        pairs = [(a, b) for ai, a in enumerate(ids) for b in ids[ai + 1:] if live[a] & live[b]]
        if pairs and dims is not None:
            pairs.sort(key=lambda ab: float(np.prod([dims[l] for l in live[ab[0]] | live[ab[1]]])))
            pairs = pairs[:k]
        a, b = rng.choice(pairs) if pairs else tuple(rng.sample(ids, 2))
        if rng.random() < 0.5:
            a, b = b, a
        path.append((a, b))
        live[nxt] = live.pop(a) | live.pop(b)
        nxt += 1
    return path


@pytest.mark.parametrize("exec_mode", EXECS)
def test_path_independence(exec_mode):
    """Greedy, operand-swapped greedy and random connected paths agree.
    Random paths are drawn among the cheapest few pairs at each step, under
    an intermediate cap of 2^22 elements; a path above the cap (HTN_E_OOM)
    or one the fused kernel cannot hold (HTN_E_UNSUPPORTED) is skipped, but
    six random paths must run on each executor."""
    rng = random.Random(7)
    w = configs.grid_network(4)
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = float(hi) + float(lo)
    net = create(w, exec_mode=exec_mode)
    greedy, _ = htn.htn_get_path(net)
    for p in (greedy, [(b, a) for a, b in greedy]):
        got = float(run(w, exec_mode=exec_mode, path=p))
        assert abs(got - ref) <= REL_F64 * abs(ref), (p, got, ref)
    ran = 0
    for _ in range(60):
        p = _random_connected_path(w.labels, rng, dims=w.dims)
        n = create(w, exec_mode=exec_mode)
        htn.htn_set_option(n, htn.HTN_OPT_MAX_INTERMEDIATE, 1 << 22)
        try:
            htn.htn_set_path(n, p)
            got = float(contract(n, ()))
        except htn.HtnError as e:
            assert e.name in ("HTN_E_OOM", "HTN_E_UNSUPPORTED")
            continue
        assert abs(got - ref) <= REL_F64 * abs(ref), (p, got, ref)
        ran += 1
        if ran == 6:
            break
    assert ran == 6, ran


def test_batch_equals_single_and_oracle():
    import torch
    ws = [configs.grid_network(s) for s in range(48)]
    nets = [create(w) for w in ws]
    outs = [htn.new_output(n) for n in nets]
    htn.htn_contract_batch(nets, outs)
    torch.cuda.synchronize()
    for w, n, o in zip(ws, nets, outs):
        single = htn.new_output(n)
        htn.htn_contract(n, single)
        torch.cuda.synchronize()
        if htn.htn_get_info(n).mults <= 2 ** 20:
            assert float(o.item()) == float(single.item())   # same plan, same kernel
        else:  # heavy nets run step by step in a batch
            assert abs(float(o.item()) - float(single.item())) <= REL_F64 * abs(float(single.item()))
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        assert abs(float(o.item()) - ref) <= REL_F64 * abs(ref)


def test_batch_graph_replays_match_eager():
    import torch
    ws = [configs.grid_network(100 + s) for s in range(32)]
    nets = [create(w) for w in ws]
    outs = [htn.new_output(n) for n in nets]
    b = htn.htn_batch_create(nets)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        htn.htn_batch_run(b, outs, stream)
    stream.synchronize()
    eager = [float(o.item()) for o in outs]
    htn.htn_batch_set_graph(b, True)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            htn.htn_batch_run(b, outs, stream)
        stream.synchronize()
        assert [float(o.item()) for o in outs] == eager, rep
    t = htn.htn_batch_timestamps(b)
    assert (t[:, 0] >= 0).all() and (t[:, 1] > t[:, 0]).all()


def test_ring_of_rings_f64():
    for seed in range(2):
        w = configs.ring_of_rings(seed)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        for exec_mode in (htn.HTN_EXEC_STEPS, htn.HTN_EXEC_AUTO):
            got = float(run(w, exec_mode=exec_mode))
            assert abs(got - ref) <= REL_F64 * abs(ref), (seed, exec_mode, got, ref)


def test_marginal_small_full_compare():
    w = configs.marginal_network(3, out_bits=6)
    ref, _ = oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
    for exec_mode in EXECS:
        got = run(w, exec_mode=exec_mode)
        assert np.abs(got - ref).max() <= 1e-15
        assert abs(got.sum() - 1.0) < 1e-12


def test_marginal_full_size_sampled_entries():
    """4096 x 4096 marginal: 64 sampled entries recomputed one by one by the
    naive oracle on sliced tensors, plus the sum invariant."""
    w = configs.marginal_network(0, out_bits=12)
    got = run(w)
    assert got.shape == (4096, 4096)
    assert abs(got.sum() - 1.0) < 1e-9
    rng = np.random.default_rng(0)
    c = 4
    for _ in range(64):
        x1, x2 = (int(v) for v in rng.integers(0, 4096, size=2))
        t1 = w.tensors[0][..., x1]
        t2 = w.tensors[1][..., x2]
        labels = [list(range(c)), list(range(c, 2 * c))] + w.labels[2:]
        ref, _ = oracle.naive_contract([t1, t2] + w.tensors[2:], labels, w.dims[:2 * c], [])
        assert abs(got[x1, x2] - float(ref)) <= 1e-17 + 1e-12 * abs(float(ref))


def test_update_data_reuses_plan():
    w = configs.grid_network(9)
    net = create(w, on_device=False)
    a = float(contract(net, ()))
    w2 = configs.grid_network(9)
    w2.tensors = [t * 0.5 if k == 0 else t for k, t in enumerate(w2.tensors)]
    htn.htn_update_data(net, [np.ascontiguousarray(t) for t in w2.tensors])
    b = float(contract(net, ()))
    assert abs(b - 0.5 * a) <= 1e-13 * abs(a)


@pytest.mark.parametrize("threads,lds", [(64, 24576), (64, 32768), (64, 65536), (256, 20480), (512, 65536),
                                         (512, 131072), (256, 163840)])
def test_fused_block_sizes_and_budgets(threads, lds):
    """Grid networks on sampled paths, fused kernel with one wave or four
    waves per network and several LDS budgets (small budgets spill)."""
    import torch
    ws = [configs.grid_network(200 + s) for s in range(24)]
    nets = []
    for w in ws:
        n = create(w, exec_mode=htn.HTN_EXEC_FUSED)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_THREADS, threads)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, lds)
        htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, 8)
        htn.htn_set_path(n, htn.HTN_PATH_SAMPLED)
        nets.append(n)
    outs = [htn.new_output(n) for n in nets]
    htn.htn_contract_batch(nets, outs)
    torch.cuda.synchronize()
    for w, n, o in zip(ws, nets, outs):
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        assert abs(float(o.item()) - ref) <= REL_F64 * abs(ref)
        single = htn.new_output(n)
        htn.htn_contract(n, single)
        torch.cuda.synchronize()
        assert float(single.item()) == float(o.item())


def test_random_batch_mixed_executors_graph_and_stamps():
    """Random networks of uneven size (the largest run step by step on a
    second stream, the rest in the fused launch), eager and graph replays
    against the oracle, and device timestamps for every net."""
    import json

    import torch
    ws = configs.random_batch(3, n=128, dtype=np.float64)
    ws = [w for i, w in enumerate(ws) if i not in (78, 79)]  # keep the oracle's time short
    nets = [create(w) for w in ws]
    stepped = [i for i, n in enumerate(nets) if not json.loads(htn.htn_plan_json(n))["fused_batch_ok"]]
    assert len(stepped) >= 2
    refs = []
    for w in ws:
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        refs.append(float(hi) + float(lo))
    outs = [htn.new_output(n) for n in nets]
    b = htn.htn_batch_create(nets)
    htn.htn_batch_set_graph(b, True)
    stream = torch.cuda.Stream()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            htn.htn_batch_run(b, htn.pointer_array(outs), stream)
        stream.synchronize()
        for i, (o, ref) in enumerate(zip(outs, refs)):
            assert abs(float(o.item()) - ref) <= REL_F64 * abs(ref) + 1e-300, (rep, i)
        t = htn.htn_batch_timestamps(b)
        assert (t[:, 0] >= 0).all() and (t[:, 1] > t[:, 0]).all(), rep


def test_autotune_picks_a_measured_configuration_and_keeps_results():
    import torch
    ws = [configs.grid_network(900 + s) for s in range(64)]
    nets = [create(w) for w in ws]
    outs = [htn.new_output(n) for n in nets]
    threads, lds, ms = htn.htn_autotune(nets, outs)
    assert threads in (64, 256, 512) and lds in (32768, 49152, 65536, 98304, 163840) and ms > 0
    htn.htn_contract_batch(nets, outs)
    torch.cuda.synchronize()
    for w, n, o in zip(ws, nets, outs):
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = float(hi) + float(lo)
        assert abs(float(o.item()) - ref) <= REL_F64 * abs(ref)
        info = htn.htn_get_info(n)
        assert info.fused_lds_bytes <= lds


@pytest.mark.parametrize("exec_mode", EXECS)
def test_edge_case_networks(exec_mode):
    from edge_cases import edge_networks
    for name, w in edge_networks(1).items():
        ref, _ = oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
        got = run(w, exec_mode=exec_mode)
        assert np.abs(got - ref).max() <= 1e-14, name


def test_torch_allocator_holds_the_library_memory():
    """With PyTorch's caching allocator installed, a net's device buffers
    (input copies, tables, workspace) are counted by torch and returned when
    the net is destroyed; results are unchanged."""
    import torch
    w = configs.grid_network(21)
    ref = float(run(w, exec_mode=htn.HTN_EXEC_STEPS))
    htn.use_torch_allocator()
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        net = create(w, exec_mode=htn.HTN_EXEC_STEPS, on_device=False)  # host data: copied into library memory
        out = htn.new_output(net)
        htn.htn_contract(net, out)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        ws = htn.htn_get_info(net).workspace_bytes
        assert held >= ws + htn.htn_get_info(net).input_bytes, (held, ws)
        assert float(out.item()) == ref
        del out
        htn.htn_destroy(net)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    finally:
        htn.htn_set_allocator(None, None)


def test_failing_allocator_reports_oom_and_the_net_recovers():
    import torch
    w = configs.grid_network(22)
    net = create(w, exec_mode=htn.HTN_EXEC_STEPS, on_device=False)
    out = htn.new_output(net)
    htn.htn_set_allocator(lambda n: 0, lambda p: None)
    try:
        with pytest.raises(htn.HtnError) as e:
            htn.htn_contract(net, out)
        assert e.value.name == "HTN_E_OOM"
    finally:
        htn.htn_set_allocator(None, None)
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    assert abs(float(out.item()) - (hi + lo)) <= REL_F64 * abs(hi + lo)


def test_failed_graph_capture_falls_back_to_stream_launches():
    """A capture forced to fail leaves the stream usable, the batch runs
    eagerly from then on with the same results, and the state says so; a
    later graph request captures normally."""
    import torch
    ws = [configs.grid_network(300 + s) for s in range(16)] + configs.random_batch(5, n=16, dtype=np.float64)
    nets = [create(w) for w in ws]
    outs = [htn.new_output(n) for n in nets]
    ptrs = htn.pointer_array(outs)
    refs = []
    for w in ws:
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        refs.append(float(hi) + float(lo))
    b = htn.htn_batch_create(nets)
    stream = torch.cuda.Stream()
    for mode, state in ((htn.HTN_GRAPH_FORCE_FAILURE, 2), (1, 1)):
        htn.htn_batch_set_graph(b, mode)
        for rep in range(3):
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                htn.htn_batch_run(b, ptrs, stream)
            stream.synchronize()
            for i, (o, ref) in enumerate(zip(outs, refs)):
                assert abs(float(o.item()) - ref) <= REL_F64 * abs(ref) + 1e-300, (mode, rep, i)
            assert htn.htn_batch_graph_state(b) == state
        if state == 2:
            assert "forced" in htn.htn_last_error()
        # the stream is not left capturing
        x = torch.ones(4, device="cuda")
        with torch.cuda.stream(stream):
            y = x * 2
        stream.synchronize()
        assert float(y.sum()) == 8.0


def _sliced(w, div, compute=htn.HTN_F64, final_sum=htn.HTN_SUM_PLAIN):
    net = create(w, compute=compute, final_sum=final_sum, storage=htn.HTN_F64)
    peak = htn.htn_get_info(net).peak_elements
    cap = max(1, int(peak // div))
    htn.htn_set_option(net, htn.HTN_OPT_SLICE, 1)
    htn.htn_set_option(net, htn.HTN_OPT_MAX_INTERMEDIATE, cap)
    info = htn.htn_get_info(net)
    labels, n_slices = htn.htn_get_slicing(net)
    assert n_slices > 1 and labels and info.n_slices == n_slices and info.peak_elements <= cap
    return net, labels


@pytest.mark.parametrize("compute,final_sum", [(htn.HTN_F64, htn.HTN_SUM_PLAIN),
                                               (htn.HTN_F64, htn.HTN_SUM_COMPENSATED),
                                               (htn.HTN_F32, htn.HTN_SUM_FP64)])
def test_sliced_contraction_matches_oracle(compute, final_sum):
    """Nets whose path exceeds an intermediate cap: the library slices summed
    labels until the path fits, contracts every slice (one batch) and sums
    them in FP64.  FP64 within 1e-10 relative of the oracle (scalars) or
    1e-14 absolute (marginal entries); FP32 within gamma(300, 2^-24) times
    the |entries| contraction.  The oracle's own slice sum over the same
    labels equals the unsliced value."""
    import torch
    cases = [(configs.grid_network(3), 20), (configs.ring_of_rings(0), 3),
             (configs.marginal_network(1, out_bits=4), 16)]
    for w, div in cases:
        net, labels = _sliced(w, div, compute, final_sum)
        shape = tuple(w.dims[l] for l in w.out_labels)
        got = contract(net, shape)
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        ref = hi + lo
        if compute == htn.HTN_F64:
            if shape:
                assert np.abs(got - ref).max() <= 1e-14, labels
            else:
                assert abs(float(got) - float(ref)) <= REL_F64 * abs(float(ref)), (labels, float(got), float(ref))
        else:
            ahi, alo = oracle.ve_contract([np.abs(t) for t in w.tensors], w.labels, w.dims, w.out_labels)
            u = 2.0 ** -24
            assert np.all(np.abs(got - ref) <= (300 * u / (1 - 300 * u)) * (ahi + alo)), labels
        if compute == htn.HTN_F64 and final_sum == htn.HTN_SUM_PLAIN and len(labels) <= 3:
            sl = oracle.sliced_contract(w.tensors, w.labels, w.dims, w.out_labels, labels)
            assert np.abs(sl - ref).max() <= 1e-13 * max(1.0, float(np.abs(ref).max()))


def test_sliced_net_is_refused_by_batches_and_noalloc_but_contracts_again():
    import torch
    w = configs.grid_network(8)
    net, _ = _sliced(w, 10)
    with pytest.raises(htn.HtnError) as e:
        htn.htn_batch_create([net])
    assert e.value.name == "HTN_E_UNSUPPORTED"
    out = htn.new_output(net)
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    with pytest.raises(htn.HtnError) as e:
        htn.htn_contract_noalloc(net, out)
    assert e.value.name == "HTN_E_UNSUPPORTED"
    a = float(out.item())
    # new data, same structure: the slices are cut again from the new inputs
    w2 = configs.grid_network(8)
    w2.tensors = [t * 2.0 if k == 0 else t for k, t in enumerate(w2.tensors)]
    htn.htn_update_data(net, [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in w2.tensors])
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    assert abs(float(out.item()) - 2.0 * a) <= 1e-13 * abs(a)
    # slicing off while the cap still binds is refused (and changes nothing)
    with pytest.raises(htn.HtnError) as e:
        htn.htn_set_option(net, htn.HTN_OPT_SLICE, 0)
    assert e.value.name == "HTN_E_OOM"
    assert htn.htn_get_slicing(net)[1] > 1
    # lift the cap (the path then fits: no slices), then slicing off
    htn.htn_set_option(net, htn.HTN_OPT_MAX_INTERMEDIATE, 2 ** 31 - 1)
    htn.htn_set_option(net, htn.HTN_OPT_SLICE, 0)
    assert htn.htn_get_slicing(net) == ([], 1)
    htn.htn_contract(net, out)
    torch.cuda.synchronize()
    assert abs(float(out.item()) - 2.0 * a) <= 1e-13 * abs(a)
