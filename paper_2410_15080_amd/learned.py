"""Training data for the learned path selector: step features paired with
measured step durations, and a helper that trains the cost model on them.

Only orchestration lives here: features come from htn_step_features, the
durations from the fused kernel's own phase clock (htn_batch_step_times),
and training runs in the library's GPU kernels (htn_model_train).
"""

from __future__ import annotations

import numpy as np

from . import htn

# Path variants used to diversify the training set: (sampled candidates,
# sampler seed); 0 candidates = FLOP-greedy.
DEFAULT_VARIANTS = ((0, 0), (1, 1), (2, 2), (4, 3), (8, 4), (32, 5))


def collect_step_timings(nets, variants=DEFAULT_VARIANTS, runs=3, max_phases=128, stream=None):
    """Run the nets as one fused batch per path variant with phase timing on.

    Returns (features [k, HTN_MODEL_FEATURES] float32, durations [k] in
    microseconds, the median over `runs` timed runs).  The nets are left on
    the FLOP-greedy path."""
    import torch
    outs = [htn.new_output(n) for n in nets]
    ptrs = htn.pointer_array(outs)
    xs, ts = [], []
    for samples, seed in variants:
        for n in nets:
            if samples == 0:
                htn.htn_set_path(n, htn.HTN_PATH_GREEDY)
            else:
                htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, samples)
                htn.htn_set_option(n, htn.HTN_OPT_PATH_SEED, seed)
                htn.htn_set_path(n, htn.HTN_PATH_SAMPLED)
        feats = [htn.htn_step_features(n) for n in nets]
        cap = max(1, max(f.shape[0] for f in feats))
        b = htn.htn_batch_create(nets)
        htn.htn_batch_set_phase_timing(b, max_phases)
        st = stream if stream is not None else torch.cuda.current_stream()
        htn.htn_batch_run(b, ptrs, st)  # warm-up
        st.synchronize()
        samples_t = []
        for _ in range(runs):
            htn.htn_batch_run(b, ptrs, st)
            st.synchronize()
            samples_t.append(htn.htn_batch_step_times(b, cap))
        tm = np.median(np.stack(samples_t), axis=0)
        for i, f in enumerate(feats):
            for q in range(f.shape[0]):
                if np.isfinite(tm[i, q]) and tm[i, q] > 0:
                    xs.append(f[q])
                    ts.append(tm[i, q])
        htn.htn_batch_destroy(b)
    for n in nets:
        htn.htn_set_path(n, htn.HTN_PATH_GREEDY)
    return np.asarray(xs, dtype=np.float32).reshape(-1, htn.HTN_MODEL_FEATURES), np.asarray(ts, dtype=np.float32)


def train_cost_model(features, durations_us, epochs=300, batch=256, lr=2e-3, seed=0, model=None):
    """Fit log(duration) with htn_model_train on the GPU.  Returns (model,
    per-epoch losses)."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(features, dtype=np.float32)).cuda()
    t = torch.from_numpy(np.log(np.asarray(durations_us, dtype=np.float64)).astype(np.float32)).cuda()
    model = model if model is not None else htn.htn_model_create(seed)
    losses = htn.htn_model_train(model, x, t, epochs, batch, lr, seed)
    return model, losses


def predict_log_us(model, features):
    """Model predictions (natural log of microseconds) for host feature rows."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(features, dtype=np.float32)).cuda()
    y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    htn.htn_model_forward(model, x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def save_model(model, path):
    """Write the model's parameters (htn_model_get_params) to an .npz file."""
    np.savez(path, params=htn.htn_model_get_params(model), features=htn.HTN_MODEL_FEATURES,
             hidden=htn.HTN_MODEL_HIDDEN)


def load_model(path, seed=0):
    """A model on the current device with the parameters saved by save_model
    (a file of another feature or hidden-layer size is refused)."""
    with np.load(path, allow_pickle=False) as f:
        if int(f["features"]) != htn.HTN_MODEL_FEATURES or int(f["hidden"]) != htn.HTN_MODEL_HIDDEN:
            raise ValueError("model file has another shape")
        params = f["params"]
    m = htn.htn_model_create(seed)
    htn.htn_model_set_params(m, params)
    return m


def save_autotune(path, threads, lds_bytes, ms, workload):
    """Record an htn_autotune choice (JSON) for reuse by later runs."""
    import json
    with open(path, "w") as f:
        json.dump({"workload": workload, "threads": int(threads), "lds_bytes": int(lds_bytes), "ms": float(ms)}, f)


def load_autotune(path, workload):
    """(threads, lds_bytes) of a saved choice for `workload`, or None."""
    import json
    import os
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("workload") != workload:
        return None
    return int(rec["threads"]), int(rec["lds_bytes"])
