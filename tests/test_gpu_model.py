"""Cost-model kernels (forward, backward, Adam) against the FP64 oracle, and
the learned path selector end to end on grid networks."""

import time

import numpy as np
import pytest

from oracle import mlp as mlp_ref
from paper_2410_15080_amd import htn
from workloads import configs

pytestmark = pytest.mark.gpu


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1.5, (n, htn.HTN_MODEL_FEATURES)).astype(np.float32)
    X[:, 10:22] = rng.integers(0, 2, (n, 12))  # flag-like columns
    t = rng.normal(1.0, 0.7, n).astype(np.float32)
    return X, t


def _model(seed=0):
    m = htn.htn_model_create(seed)
    return m, htn.htn_model_get_params(m).astype(np.float64)


def test_init_is_seeded_he_uniform():
    m1, p1 = _model(7)
    m2, p2 = _model(7)
    _, p3 = _model(8)
    assert np.array_equal(p1, p2) and not np.array_equal(p1, p3)
    W1, b1, W2, b2, w3, b3 = mlp_ref.unpack(p1)
    assert np.abs(W1).max() <= np.sqrt(6 / htn.HTN_MODEL_FEATURES) and np.abs(W2).max() <= np.sqrt(6 / 64)
    assert not b1.any() and not b2.any() and b3 == 0.0


@pytest.mark.parametrize("n", [1, 255, 1000])
def test_forward_matches_oracle(n):
    import torch
    m, p = _model(1)
    X, _ = _data(n, n)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    htn.htn_model_forward(m, torch.from_numpy(X).cuda(), y)
    torch.cuda.synchronize()
    ref, _ = mlp_ref.forward(p, X.astype(np.float64))
    # FP32 arithmetic over ~5.6e3 multiply-adds per sample
    np.testing.assert_allclose(y.cpu().numpy(), ref, rtol=1e-4, atol=1e-4)


def test_gradients_match_oracle():
    import torch
    m, p = _model(2)
    X, t = _data(3, 512)
    g = torch.empty(htn.htn_model_param_count(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    htn.htn_model_gradients(m, torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(), g, loss)
    torch.cuda.synchronize()
    ref = mlp_ref.gradients(p, X.astype(np.float64), t.astype(np.float64))
    got = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
    assert float(loss.item()) == pytest.approx(mlp_ref.loss(p, X, t), rel=1e-5)


def test_gradients_are_bit_reproducible():
    import torch
    m, _ = _model(4)
    X, t = _data(5, 300)
    x, tt = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    g1 = torch.empty(htn.htn_model_param_count(), dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    htn.htn_model_gradients(m, x, tt, g1)
    htn.htn_model_gradients(m, x, tt, g2)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_adam_steps_match_oracle():
    import torch
    m, p = _model(6)
    rng = np.random.default_rng(6)
    mm, vv = np.zeros_like(p), np.zeros_like(p)
    lr = 1e-3
    for k in range(1, 4):
        g = rng.normal(size=p.size).astype(np.float32)
        htn.htn_model_adam_step(m, torch.from_numpy(g).cuda(), lr)
        p, mm, vv = mlp_ref.adam_step(p, mm, vv, g.astype(np.float64), lr, k)
    got = htn.htn_model_get_params(m).astype(np.float64)
    np.testing.assert_allclose(got, p, rtol=0, atol=1e-6)


def test_training_fits_a_teacher_and_is_deterministic():
    import torch
    X, _ = _data(9, 4096)
    teacher = htn.htn_model_create(123)
    x = torch.from_numpy(X).cuda()
    t = torch.empty(4096, dtype=torch.float32, device="cuda")
    htn.htn_model_forward(teacher, x, t)
    finals = []
    for _ in range(2):
        s = htn.htn_model_create(5)
        losses = htn.htn_model_train(s, x, t, 60, 256, 3e-3, seed=11)
        finals.append(htn.htn_model_get_params(s))
        assert np.all(np.isfinite(losses))
        assert losses[-1] < 0.05 * losses[0], losses[[0, -1]]
    assert np.array_equal(finals[0], finals[1])


def test_step_times_cover_every_fused_step():
    import torch
    ws = [configs.grid_network(700 + s) for s in range(16)]
    nets = [htn.htn_create([torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in w.tensors], w.labels,
                           w.dims, w.out_labels) for w in ws]
    for n in nets:
        htn.htn_set_path(n, htn.HTN_PATH_SAMPLED)
    outs = [htn.new_output(n) for n in nets]
    b = htn.htn_batch_create(nets)
    htn.htn_batch_set_phase_timing(b, 128)
    htn.htn_batch_run(b, htn.pointer_array(outs))
    torch.cuda.synchronize()
    k = [htn.htn_get_info(n).n_kernel_steps for n in nets]
    tm = htn.htn_batch_step_times(b, max(k) + 2)
    se = htn.htn_batch_timestamps(b)
    import json
    for i, ki in enumerate(k):
        plan = json.loads(htn.htn_plan_json(nets[i]))
        phases = {}
        for st in plan["steps"]:
            if not st["absorbed"]:
                phases[st["f_phase"]] = phases.get(st["f_phase"], 0) + 1
        rec = tm[i, :ki]
        # one recorded duration per phase (its heaviest step), the rest NaN
        assert int(np.isfinite(rec).sum()) == len(phases) and np.all(rec[np.isfinite(rec)] > 0)
        assert np.all(np.isnan(tm[i, ki:]))
        # phases are disjoint intervals inside the network's run
        assert np.nansum(rec) <= (se[i, 1] - se[i, 0]) * 0.01 + 1e-3
        assert htn.htn_step_features(nets[i]).shape == (ki, htn.HTN_MODEL_FEATURES)


def test_step_times_cover_nets_run_step_by_step():
    """Nets forced onto the per-step executor get one duration per kernel
    step from clock reads between their launches; together they span the
    net's run."""
    import torch
    ws = [configs.grid_network(900 + s) for s in range(6)]
    nets = [htn.htn_create([torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in w.tensors], w.labels,
                           w.dims, w.out_labels) for w in ws]
    for n in nets[:3]:
        htn.htn_set_option(n, htn.HTN_OPT_EXEC, htn.HTN_EXEC_STEPS)
    outs = [htn.new_output(n) for n in nets]
    b = htn.htn_batch_create(nets)
    htn.htn_batch_set_phase_timing(b, 64)
    htn.htn_batch_run(b, htn.pointer_array(outs))
    torch.cuda.synchronize()
    k = [htn.htn_get_info(n).n_kernel_steps for n in nets]
    tm = htn.htn_batch_step_times(b, max(k))
    se = htn.htn_batch_timestamps(b)
    for i in range(3):
        rec = tm[i, :k[i]]
        assert np.all(np.isfinite(rec)) and np.all(rec > 0)
        assert rec.sum() <= (se[i, 1] - se[i, 0]) * 0.01 + 1e-3
        assert htn.htn_step_features(nets[i])[:, 21].max() == 0.0  # per-step executor rows
    import oracle
    for w, o in zip(ws, outs):
        hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
        assert abs(float(o[0].item()) - (hi + lo)) <= 1e-10 * max(1.0, abs(hi + lo))


def _batch_ms(nets, reps=20):
    import torch
    outs = [htn.new_output(n) for n in nets]
    ptrs = htn.pointer_array(outs)
    b = htn.htn_batch_create(nets)
    st = torch.cuda.current_stream()
    for _ in range(3):
        htn.htn_batch_run(b, ptrs, st)
    st.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        htn.htn_batch_run(b, ptrs, st)
    st.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    res = np.array([float(o[0].item()) for o in outs])
    htn.htn_batch_destroy(b)
    return ms, res


def _median_ms(nets, reps=7):
    """Median and spread (max - min) of `reps` batch timings of 20 runs."""
    ms, res = [], None
    for _ in range(reps):
        m, res = _batch_ms(nets)
        ms.append(m)
    return float(np.median(ms)), float(max(ms) - min(ms)), res


def _constant_model(log_us=np.log(10.0)):
    """A model whose every prediction is the same (all weights 0, output
    bias log_us): it ranks candidates by their count of fused phases."""
    m = htn.htn_model_create(0)
    p = np.zeros(htn.htn_model_param_count(), dtype=np.float32)
    p[-1] = log_us
    htn.htn_model_set_params(m, p)
    return m


def test_learned_paths_beat_flop_greedy_on_grid_batches():
    """Train on timings of one set of grid networks, select paths for a
    held-out set, and compare measured batch times (median of seven timings
    of 20 runs each) against FLOP-greedy orders, the FLOP-cheapest sampled
    candidate, and the same selector driven by two control models: the
    untrained network (random weights) and a constant prediction (which
    ranks candidates by their number of fused phases).  Results must not
    change with the path."""
    import json as _json
    import torch
    from paper_2410_15080_amd import learned

    def make(seeds):
        ws = [configs.grid_network(s) for s in seeds]
        return ws, [htn.htn_create([torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in w.tensors],
                                   w.labels, w.dims, w.out_labels) for w in ws]

    _, train = make(range(20000, 20128))
    X, t = learned.collect_step_timings(train, runs=2)
    assert X.shape[0] > 1000
    model, losses = learned.train_cost_model(X, t, epochs=150, batch=256, lr=2e-3, seed=0)
    assert losses[-1] < 0.5 * losses[0]

    ws, test = make(range(256))
    greedy_ms, greedy_spread, greedy_res = _median_ms(test)
    for n in test:
        htn.htn_set_path(n, htn.HTN_PATH_SAMPLED)
    sampled_ms, sampled_spread, _ = _median_ms(test)
    timings = {}
    for name, m in (("untrained", htn.htn_model_create(7)), ("constant", _constant_model()), ("trained", model)):
        for n in test:
            htn.htn_set_model(n, m)
            htn.htn_set_path(n, htn.HTN_PATH_LEARNED)
        ms, spread, res = _median_ms(test)
        np.testing.assert_allclose(res, greedy_res, rtol=1e-10, atol=1e-15)
        timings[name] = (ms, spread)
    learned_ms, learned_spread = timings["trained"]
    print("learned-path timings (ms, spread): " + _json.dumps(
        {"greedy": (greedy_ms, greedy_spread), "sampled_flop_best": (sampled_ms, sampled_spread), **timings}))
    assert learned_ms < 0.8 * greedy_ms
    # what training adds: faster than both control models by more than the
    # spread of the timings
    noise = max(learned_spread, timings["untrained"][1], timings["constant"][1])
    assert learned_ms + noise < timings["untrained"][0], timings
    assert learned_ms + noise < timings["constant"][0], timings
    # and no slower than the FLOP proxy beyond the timing spread
    assert learned_ms <= sampled_ms + max(learned_spread, sampled_spread), (learned_ms, sampled_ms)


def test_learned_path_without_model_is_greedy():
    import torch
    w = configs.grid_network(3)
    n = htn.htn_create([torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in w.tensors], w.labels, w.dims,
                       w.out_labels)
    g = htn.htn_get_path(n)
    htn.htn_set_path(n, htn.HTN_PATH_LEARNED)
    assert htn.htn_get_path(n) == g


def test_model_and_autotune_choice_persist(tmp_path):
    from paper_2410_15080_amd import learned
    import torch
    m = htn.htn_model_create(11)
    p = htn.htn_model_get_params(m)
    learned.save_model(m, str(tmp_path / "m.npz"))
    m2 = learned.load_model(str(tmp_path / "m.npz"))
    assert np.array_equal(htn.htn_model_get_params(m2), p)
    x = torch.rand(32, htn.HTN_MODEL_FEATURES, device="cuda")
    y1 = torch.empty(32, device="cuda")
    y2 = torch.empty(32, device="cuda")
    htn.htn_model_forward(m, x, y1)
    htn.htn_model_forward(m2, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    learned.save_autotune(str(tmp_path / "t.json"), 256, 65536, 0.5, "grid")
    assert learned.load_autotune(str(tmp_path / "t.json"), "grid") == (256, 65536)
    assert learned.load_autotune(str(tmp_path / "t.json"), "ring") is None
