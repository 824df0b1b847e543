"""Host-side checks of the C ABI: the library loads, exports what the header
declares, validates structure, and accounts cost exactly like the oracle's
cost model.  Nothing here touches a GPU (htn_create with host data and
path planning make no HIP call)."""

import json
import os
import random

import numpy as np
import pytest

import oracle
from paper_2410_15080_amd import htn
from workloads import configs

import circuit_nets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_declared_symbol():
    lib = htn.load_library()
    declared = htn.declared_symbols()
    assert len(declared) >= 17
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    for code, name in enumerate(htn.STATUS):
        assert htn.htn_status_string(code) == name


def _host_net(net_w, **kw):
    return htn.htn_create(net_w.tensors, net_w.labels, net_w.dims, net_w.out_labels, **kw)


def test_worked_example_paths_and_costs():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    rng = np.random.default_rng(0)
    ts = [rng.uniform(-1, 1, size=[g["dims"][l] for l in ls]) for ls in g["labels"]]
    net = htn.htn_create(ts, g["labels"], g["dims"], [])
    htn.htn_set_path(net, g["path"])
    path, mults = htn.htn_get_path(net)
    assert path == [tuple(p) for p in g["path"]]
    assert mults == g["expected_total"]
    # FLOP-greedy never does worse than the printed order here
    htn.htn_set_path(net, htn.HTN_PATH_GREEDY)
    gpath, gm = htn.htn_get_path(net)
    assert gm <= g["expected_total"]
    assert gm == sum(oracle.path_cost(g["labels"], g["dims"], [], gpath))


def _random_ssa_path(labels, rng):
    """A random valid SSA path (any pair order, connected or not)."""
    live = list(range(len(labels)))
    nxt = len(labels)
    path = []
    while len(live) > 1:
        i, j = rng.sample(live, 2)
        path.append((i, j))
        live.remove(i)
        live.remove(j)
        live.append(nxt)
        nxt += 1
    return path


@pytest.mark.parametrize("maker", ["grid", "ring", "gates"])
def test_planner_cost_matches_oracle_cost_model(maker):
    rng = random.Random(3)
    for seed in range(4):
        if maker == "grid":
            w = configs.grid_network(seed)
        elif maker == "ring":
            w = configs.ring_of_rings(seed)
        else:
            w, _ = circuit_nets.cut_gates(seed, 2)
        net = _host_net(w)
        path, m = htn.htn_get_path(net)
        assert m == sum(oracle.path_cost(w.labels, w.dims, w.out_labels, path))
        if maker == "gates":
            rp = _random_ssa_path(w.labels, rng)
            htn.htn_set_path(net, rp)
            _, m2 = htn.htn_get_path(net)
            assert m2 == sum(oracle.path_cost(w.labels, w.dims, w.out_labels, rp))


def test_random_paths_on_small_networks_match_cost_model():
    rng = random.Random(5)
    nrng = np.random.default_rng(5)
    for _ in range(40):
        n_labels = int(nrng.integers(3, 7))
        dims = [int(d) for d in nrng.integers(2, 5, size=n_labels)]
        labels = [[int(x) for x in nrng.choice(n_labels, size=int(nrng.integers(1, 4)), replace=False)]
                  for _ in range(int(nrng.integers(2, 6)))]
        used = sorted({l for ls in labels for l in ls})
        out = [int(x) for x in nrng.choice(used, size=min(len(used), int(nrng.integers(0, 3))), replace=False)]
        ts = [nrng.uniform(-1, 1, size=[dims[l] for l in ls]) for ls in labels]
        net = htn.htn_create(ts, labels, dims, out)
        rp = _random_ssa_path(labels, rng)
        htn.htn_set_path(net, rp)
        _, m = htn.htn_get_path(net)
        assert m == sum(oracle.path_cost(labels, dims, out, rp))


def test_absorption_folds_coefficient_vectors():
    w = configs.grid_network(0)
    net = _host_net(w)
    info = htn.htn_get_info(net)
    assert info.n_absorbed == 24          # every CT folds into a QT load
    assert info.n_kernel_steps == 15      # 16 QTs -> 15 pairwise kernels
    plan = json.loads(htn.htn_plan_json(net))
    assert sum(1 for s in plan["steps"] if s["absorbed"]) == 24


def test_marginal_plan_is_one_big_contraction():
    w = configs.marginal_network(0, out_bits=12)
    net = _host_net(w)
    plan = json.loads(htn.htn_plan_json(net))
    last = plan["steps"][-1]
    assert last["final"] and last["n_out"] == 4096 * 4096 and last["n_sum"] == 256
    assert plan["mults"] == 4 * 4 ** 5 * 4096 + 4096 * 4096 * 256


def _expect(status, fn, *a, **kw):
    with pytest.raises(htn.HtnError) as e:
        fn(*a, **kw)
    assert e.value.name == status, str(e.value)


def test_structural_errors():
    a = np.ones((2, 3))
    b = np.ones((3, 4))
    _expect("HTN_E_LABEL", htn.htn_create, [a, b], [[0, 1], [1, 5]], [2, 3, 4], [])
    _expect("HTN_E_LABEL", htn.htn_create, [np.ones((2, 2))], [[0, 0]], [2, 3], [])
    _expect("HTN_E_LABEL", htn.htn_create, [a, b], [[0, 1], [1, 2]], [2, 3, 4, 5], [3])
    _expect("HTN_E_LABEL", htn.htn_create, [a, b], [[0, 1], [1, 2]], [2, 3, 4], [0, 0])
    net = htn.htn_create([a, b], [[0, 1], [1, 2]], [2, 3, 4], [0, 2])
    _expect("HTN_E_PATH", htn.htn_set_path, net, [(0, 0)])
    _expect("HTN_E_PATH", htn.htn_set_path, net, [(0, 2)])
    _expect("HTN_E_PATH", htn.htn_set_path, net, [(0, 1), (2, 0)])
    _expect("HTN_E_ARG", htn.htn_set_path, net, -7)
    _expect("HTN_E_ARG", htn.htn_set_option, net, htn.HTN_OPT_EXEC, 9)
    _expect("HTN_E_ARG", htn.htn_set_option, net, htn.HTN_OPT_QUEUE, 3)
    _expect("HTN_E_ARG", htn.htn_set_option, net, htn.HTN_OPT_QUEUE, -1)
    for mode in (0, 1, 2):
        htn.htn_set_option(net, htn.HTN_OPT_QUEUE, mode)
    # a failed call leaves the previous path in place
    htn.htn_set_path(net, [(1, 0)])
    _expect("HTN_E_PATH", htn.htn_set_path, net, [(1, 1)])
    assert htn.htn_get_path(net)[0] == [(1, 0)]


def test_intermediate_cap_reports_oom():
    w = configs.marginal_network(0, out_bits=8)
    net = _host_net(w)
    _expect("HTN_E_OOM", htn.htn_set_option, net, htn.HTN_OPT_MAX_INTERMEDIATE, 1000)
    # the previous plan survives
    assert htn.htn_get_info(net).out_elements == 256 * 256


def test_output_dtype_follows_final_sum():
    w = configs.grid_network(0)
    for compute, fs, want in [(htn.HTN_F64, htn.HTN_SUM_PLAIN, htn.HTN_F64),
                              (htn.HTN_F32, htn.HTN_SUM_PLAIN, htn.HTN_F32),
                              (htn.HTN_F32, htn.HTN_SUM_COMPENSATED, htn.HTN_F64),
                              (htn.HTN_BF16, htn.HTN_SUM_FP64, htn.HTN_F64)]:
        net = _host_net(w, compute=compute, final_sum=fs)
        assert htn.htn_get_info(net).out_dtype == want


def test_qpd_sampler_host_logic_matches_oracle():
    # htn_qpd_sample is host code (no device call): draws and weights equal
    # the oracle's on the same uniforms
    from oracle import qpd_sampling as qs
    rng = np.random.default_rng(9)
    for c in (np.array([0.5, 0.5, 0.5, -0.5, 0.5, -0.5]), np.array([0.0, 2.5, -0.1, 0.0, -3.0])):
        for s in (1, 5, 4096):
            u = rng.random(s)
            n, w = htn.htn_qpd_sample(c, s, u)
            assert np.array_equal(n, qs.sample_counts(c, s, u))
            assert np.array_equal(w, qs.estimator_weights(c, n, s))


def test_truncation_items_are_validated_before_any_device_call():
    for kept, dims in (([[0, 6], None], (6, 4)), ([[], None], (6, 4)), ([None, None], (6, 0))):
        with pytest.raises(htn.HtnError, match="HTN_E_ARG"):
            htn.htn_truncate_create([(1, 2, dims, kept)], htn.HTN_F64)


def test_noalloc_rejects_a_workspace_above_its_limit_on_the_host():
    """Three 4096 x 4096 matrices in a chain: the per-step workspace holds a
    128 MiB intermediate, above the allocation-free limit; the call fails on
    the host before touching a device."""
    import numpy as np
    from paper_2410_15080_amd import htn
    d = 4096
    ts = [np.zeros((d, d)), np.zeros((d, d)), np.zeros((d, d))]
    net = htn.htn_create(ts, [[0, 1], [1, 2], [2, 3]], [d, d, d, d], [0, 3])
    info = htn.htn_get_info(net)
    assert info.workspace_bytes > htn.HTN_NOALLOC_SCRATCH_BYTES
    with pytest.raises(htn.HtnError) as e:
        htn.htn_contract_noalloc(net, np.zeros(1))  # rejected before the output is used
    assert e.value.name == "HTN_E_UNSUPPORTED"


def test_allocator_hook_arguments_are_checked_on_the_host():
    import ctypes
    from paper_2410_15080_amd import htn
    lib = htn.load_library()
    fn = htn.ALLOC_FN(lambda n, c: None)
    assert lib.htn_set_allocator(ctypes.cast(fn, ctypes.c_void_p), None, None) == 1  # HTN_E_ARG
    assert lib.htn_set_allocator(None, None, None) == 0


def test_qt_evaluator_validates_on_the_host():
    from paper_2410_15080_amd import htn
    init = np.array([[1.0, 0.0, 0.0, 0.0]] * 2)
    bad = [
        [(2, init, [], "ZQ", [])],                         # observable letter
        [(2, init, [], "ZI", [0])],                        # kept qubit not I
        [(2, init, [(htn.HTN_SV_CZ, 0, 0, [0] * 8)], "ZZ", [])],  # CZ on one qubit
        [(2, init, [(htn.HTN_SV_PROJ, 0, 2, [0] * 8)], "ZZ", [])],  # projection bit
        [(25, np.zeros((25, 4)), [], "I" * 25, [])],       # too many qubits
    ]
    for insts in bad:
        with pytest.raises(htn.HtnError) as e:
            htn.htn_qt_eval_create(insts, np.array([0, 1]), np.array([0]), np.array([1.0]))
        assert e.value.name == "HTN_E_ARG"
    with pytest.raises(htn.HtnError) as e:   # term output beyond the outputs
        htn.htn_qt_eval_create([(2, init, [], "ZZ", [])], np.array([0, 1]), np.array([1]), np.array([1.0]))
    assert e.value.name == "HTN_E_ARG"
