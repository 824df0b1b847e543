"""Host replay of libhtn plans against the oracle (no GPU).

The replay (tests/plan_emulator.py) executes the exact offset tables and
layouts the planner emits, for both executors.  It catches planner errors
(tables, layout choices, absorption, packing) on the CPU."""

import random

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
import circuit_nets
from plan_emulator import replay
from workloads import configs
from workloads.network import Network


def _check(w, path=None, lds=None, threads=None):
    net = htn.htn_create(w.tensors, w.labels, w.dims, w.out_labels)
    if lds is not None:
        htn.htn_set_option(net, htn.HTN_OPT_FUSED_LDS_BYTES, lds)
    if threads is not None:
        htn.htn_set_option(net, htn.HTN_OPT_FUSED_THREADS, threads)
    if path is not None:
        try:
            htn.htn_set_path(net, path)
        except htn.HtnError as e:
            assert e.name == "HTN_E_OOM"
            return
        if htn.htn_get_info(net).peak_elements > 2e6:
            return
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    ref = hi + lo
    scale = max(1e-300, float(np.abs(ref).max()))
    plan_possible = htn.htn_plan_json(net).find('"fused_possible":true') >= 0
    for ex in ("steps", "fused", "program"):
        if ex == "program" and not plan_possible:
            continue
        got = replay(w, net, ex, threads=threads or 256)
        assert float(np.abs(got - ref).max()) <= 1e-12 * scale, ex


def _random_network(rng):
    n_labels = int(rng.integers(3, 8))
    dims = [int(d) for d in rng.integers(1, 6, size=n_labels)]
    labels = []
    for _ in range(int(rng.integers(1, 6))):
        r = int(rng.integers(1, min(4, n_labels) + 1))
        labels.append([int(x) for x in rng.choice(n_labels, size=r, replace=False)])
    used = sorted({l for ls in labels for l in ls})
    out = [int(x) for x in rng.choice(used, size=min(int(rng.integers(0, 4)), len(used)), replace=False)]
    tensors = [rng.uniform(-1, 1, size=[dims[l] for l in ls]) for ls in labels]
    return Network(tensors, labels, dims, out)


@pytest.mark.parametrize("seed", range(8))
def test_replay_grid(seed):
    _check(configs.grid_network(seed))
    _check(configs.grid_network(seed), threads=64, lds=16384)
    _check(configs.grid_network(seed), threads=512, lds=131072)


def test_replay_sampled_paths():
    for seed in range(6):
        w = configs.grid_network(seed)
        net = htn.htn_create(w.tensors, w.labels, w.dims, w.out_labels)
        htn.htn_set_option(net, htn.HTN_OPT_PATH_SAMPLES, 16)
        htn.htn_set_path(net, htn.HTN_PATH_SAMPLED)
        path, _ = htn.htn_get_path(net)
        _check(w, path=path)
        _check(w, path=path, threads=64, lds=16384)
        _check(w, path=path, threads=512, lds=98304)


def test_replay_random_networks():
    rng = np.random.default_rng(11)
    for _ in range(60):
        _check(_random_network(rng))


def _random_path(w, rng):
    """A uniformly random order of steps between tensors sharing a label."""
    live = {i: set(ls) for i, ls in enumerate(w.labels)}
    nxt = len(w.labels)
    path = []
    while len(live) > 1:
        ids = sorted(live)
        pairs = [(a, b) for ai, a in enumerate(ids) for b in ids[ai + 1:] if live[a] & live[b]]
        a, b = rng.choice(pairs)
        if rng.random() < 0.5:
            a, b = b, a
        path.append((a, b))
        live[nxt] = live.pop(a) | live.pop(b)
        nxt += 1
    return path


def test_replay_random_paths():
    rng = random.Random(7)
    w = configs.grid_network(4)
    for _ in range(8):
        _check(w, _random_path(w, rng))


def test_replay_small_lds_budgets_spill():
    for lds in (4096, 16384):
        _check(configs.grid_network(5), lds=lds)


def test_replay_ring_and_marginal_and_circuits():
    _check(configs.ring_of_rings(0))
    _check(configs.marginal_network(0, out_bits=7))
    _check(circuit_nets.cut_wires(0))
    _check(circuit_nets.cut_gates(0, 2)[0])


def test_replay_random_batch_networks():
    for w in configs.random_batch(3, n=24, dtype=np.float64):
        if w.input_elements() < 300000:
            _check(w)


def test_replay_edge_cases():
    from edge_cases import edge_networks
    for name, w in edge_networks().items():
        _check(w)


def test_marginal_operands_written_in_packed_order():
    """The folds that produce the marginal's GEMM operands write them in the
    packed [M][K] / [N][K] order, so the matrix-core step needs no pack
    launch (checked as an identity permutation by the replay)."""
    import json
    w = configs.marginal_network(0, out_bits=9)  # 512 x 512 x 256: above the fused batch limit
    net = htn.htn_create(w.tensors, w.labels, w.dims, w.out_labels)
    steps = json.loads(htn.htn_plan_json(net))["steps"]
    gemm = [st for st in steps if st["mfma"]]
    assert gemm and all(st["pack_id"] == [1, 1] for st in gemm)
    _check(w)


def _qpd_grid(seed, s_qpd):
    """A grid network after QPD sampling of its gate cuts (oracle draws)."""
    from oracle import qpd_sampling as qs
    w = configs.grid_network(seed)
    rng = np.random.default_rng(1000 + seed)
    gate = [i for i, t in enumerate(w.tensors) if w.kinds[i] == "ct" and t.size == 6]
    counts = [qs.sample_counts(w.tensors[c], s_qpd, rng.random(s_qpd)) for c in gate]
    return qs.truncate(w, gate, counts, s_qpd)


@pytest.mark.parametrize("seed", range(6))
def test_one_draw_per_gate_cut_folds_scalar_factors(seed):
    """With one draw per gate cut every sampled label keeps one index, so each
    gate CT is a single number: the planner folds these scalar factors into
    input loads on any path, and the 16 QTs take 15 kernel steps (none for
    a coefficient tensor); the replayed plans equal the oracle."""
    w = _qpd_grid(seed, 1)
    for path in (htn.HTN_PATH_GREEDY, htn.HTN_PATH_SAMPLED):
        net = htn.htn_create(w.tensors, w.labels, w.dims, w.out_labels)
        htn.htn_set_option(net, htn.HTN_OPT_PATH_SAMPLES, 64)
        htn.htn_set_path(net, path)
        info = htn.htn_get_info(net)
        assert info.n_kernel_steps == 15, (path, info.n_kernel_steps)
        assert info.n_absorbed == len(w.tensors) - 16
    _check(w)
    _check(w, path=htn.htn_get_path(net)[0])
    rng = random.Random(seed)
    for _ in range(4):
        _check(w, path=_random_path(w, rng))
