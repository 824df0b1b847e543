#!/usr/bin/env python3
"""h-TN contraction throughput on one MI355X.

Default workload (one "step"): a batch of 1024 seeded 4x4-grid h-TNs -- 16
quantum tensors, 24 cuts, each cut a wire cut (dim 4, Pauli-basis weights
1/2) or a CZ gate cut (dim 6, six QPD weights) drawn 50/50 per edge, QT
entries U[-1,1] -- contracted in FP64 to each network's scalar <O>.  The
batch runs as one input-materialisation launch plus one launch of the fused
kernel (one workgroup per network).  Inputs are resident in HBM before
timing.

Other workloads (--workload), each printing one JSON line of the same form:
  random     512 random networks of uneven size (3-12 QTs, 2-14 cuts), FP32
             with an FP64 final sum, one graph launch per batch; per-network
             latency p50/p99 from device timestamps
  marginal   one 4096 x 4096 marginal: two [4]^4 x 4096 QTs joined by four
             CutQC wire tensors (a 4096 x 4096 x 256 matrix product after the
             coefficient fold), FP64 / FP32 / BF16 inputs, FP64 output
  ring       256 ring-of-rings networks (64 QTs, 3-6 cuts each), FP64 / FP32
             / BF16 with a compensated FP64 final sum

Reported:
  value        GFLOP/s = 2 * (multiplications of the FLOP-greedy paths) / time;
               the same numerator for every path variant, so a cheaper
               path shows up as higher throughput, never as extra flops
  htns_per_s   networks per second
  roofline     the dominant kernel against its bound, on the work it executes
  cpu_baseline the CPU oracle on a bounded sample of the same workload
"""

import argparse
import concurrent.futures
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64_valu": 78.6, "f32_valu": 157.3, "f64_mfma": 78.6, "f32_mfma": 157.3, "bf16_mfma": 2500.0,
        "hbm_gbs": 8000.0}
METRIC = "h-TN contraction GFLOP/s & h-TNs/s vs plain FP64 path, at stated rel. error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["grid", "random", "marginal", "ring", "qpd"],
                    default="grid")
    ap.add_argument("--batch", type=int, default=None, help="networks per batch (default per workload)")
    ap.add_argument("--dtype", choices=["f64", "f32", "bf16"], default=None)
    ap.add_argument("--lds", type=int, default=None,
                    help="fused kernel LDS budget per network in bytes (default: 81920 for grid -- two "
                         "workgroups fill a CU's 160 KiB -- and 65536 otherwise)")
    ap.add_argument("--threads", type=int, default=256, choices=[64, 256, 512])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--path", choices=["greedy", "sampled", "learned"], default=None,
                    help="contraction paths (default: sampled for grid and marginal, learned for the random "
                         "serving batch, greedy for ring)")
    ap.add_argument("--samples", type=int, default=None,
                    help="sampled path candidates per network (default: 128 for grid and random, 32 for ring)")
    ap.add_argument("--qpd-samples", type=int, default=8,
                    help="QPD draws per gate-cut CT (qpd workload)")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="measure the fused kernel's workgroup size and LDS budget first "
                         "(auto: on for the random and ring batches)")
    return ap.parse_args()


# HBM traffic per launch of a kernel on a workload, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this script scaled by the same counters
# on a plain copy (profiles/ holds the summaries and commands).  Each record
# carries a digest of the sources that shape the kernel and its plans; when
# they change the record no longer applies and traffic is reported as null.
TRAFFIC = {
    # profiles/k_fused_grid4x4_batch1024_f64.md: FETCH_SIZE 18 797.3125 x 2048 B, WRITE_SIZE 213.5 x 1024 B
    "k_fused_grid": {"read_bytes": 38_496_896, "write_bytes": 218_624, "sources": "af6e1d77f20c0f03",
                     "profile": "profiles/k_fused_grid4x4_batch1024_f64.md"},
    # profiles/k_truncate_grid4x4_qpd8_batch1024_f64.md: FETCH_SIZE 13 476 x 2048 B, WRITE_SIZE 15 552.6 x 1024 B
    "k_truncate_qpd8": {"read_bytes": 27_598_848, "write_bytes": 15_925_862, "sources": "c89d2a641b3a6971",
                        "files": ["paper_2410_15080_amd/csrc/qpd.hip", "paper_2410_15080_amd/csrc/api.hip",
                                  "paper_2410_15080_amd/csrc/kernels.hpp"],
                        "profile": "profiles/k_truncate_grid4x4_qpd8_batch1024_f64.md"},
}
TRAFFIC_SOURCES = ["paper_2410_15080_amd/csrc/fused.hpp", "paper_2410_15080_amd/csrc/kern_common.hpp",
                   "paper_2410_15080_amd/csrc/fused_b256.hip", "paper_2410_15080_amd/csrc/planner.cpp"]


def source_digest(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in files or TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key, runs_ok=True):
    rec = TRAFFIC.get(key)
    if not rec or not runs_ok or rec["sources"] != source_digest(rec.get("files")):
        return None
    return {"read_bytes": rec["read_bytes"], "write_bytes": rec["write_bytes"],
            "bytes": rec["read_bytes"] + rec["write_bytes"], "profile": rec["profile"]}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def dtype_code(name):
    from paper_2410_15080_amd import htn
    return {"f64": htn.HTN_F64, "f32": htn.HTN_F32, "bf16": htn.HTN_BF16}[name]


def cpu_baseline(ws, seconds, mults):
    """Time the oracle (FP64 variable elimination) on as many networks as fit
    in about `seconds`, one network per host thread."""
    import oracle
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    oracle.set_num_threads(1)

    def one(w):
        return float(oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels, mode="f64"))

    done = 0
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=cores) as ex:
        while time.perf_counter() - t0 < seconds and done < len(ws):
            chunk = ws[done:done + cores * 4]
            list(ex.map(one, chunk))
            done += len(chunk)
    dt = time.perf_counter() - t0
    cm = float(sum(mults[:done]))
    return {"value": 2.0 * cm / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "htns_per_s": done / dt,
            "sample": f"first {done} of the {len(ws)} networks, FP64 variable elimination, one network per "
                      f"thread, {dt:.1f} s"}


def oracle_ref(w):
    import oracle
    hi, lo = oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels)
    return float(hi) + float(lo)


class Timer:
    """Times a callable that enqueues work on `stream`: wall clock over the
    K timed calls (bracketed by synchronisation) and the mean of per-call
    HIP event intervals on the same stream."""

    def __init__(self, stream):
        self.stream = stream

    def run(self, fn, steps, warmup, after_warmup=None):
        import numpy as np
        import torch
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                fn()
        self.stream.synchronize()
        if after_warmup:
            after_warmup()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            for k in range(steps):
                ev[k][0].record(self.stream)
                fn()
                ev[k][1].record(self.stream)
        self.stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall * 1e3 / steps, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def make_nets(ws, compute, final_sum, args, path):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    dev = torch.device("cuda:0")
    tdt = {htn.HTN_F64: torch.float64, htn.HTN_F32: torch.float32, htn.HTN_BF16: torch.float32}[compute]
    storage = htn.HTN_F64 if compute == htn.HTN_F64 else htn.HTN_F32
    nets, greedy = [], []
    for w in ws:
        ts = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(dev).to(tdt) for t in w.tensors]
        n = htn.htn_create(ts, w.labels, w.dims, w.out_labels, compute=compute, final_sum=final_sum,
                           storage=storage)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, args.lds)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_THREADS, args.threads)
        greedy.append(htn.htn_get_info(n).mults)
        nets.append(n)
    if path != "greedy":
        model = None
        if path == "learned":
            model = train_model(ws, compute, final_sum, args)
        for n in nets:
            htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, args.samples)
            if model is not None:
                htn.htn_set_model(n, model)
            htn.htn_set_path(n, htn.HTN_PATH_SAMPLED if path == "sampled" else htn.HTN_PATH_LEARNED)
    return nets, greedy


def train_model(ws, compute, final_sum, args):
    """Cost model trained on step timings of a disjoint set of networks of
    the same workload (seeds offset by 10^5)."""
    from paper_2410_15080_amd import learned
    from workloads import configs
    log("training the cost model")
    kind = ws[0].meta.get("config")
    if kind == "grid":
        tws = [configs.grid_network(100000 + s) for s in range(512)]
    elif kind == "random_batch":
        tws = configs.random_batch(100000, n=512)
    else:
        tws = ws[: min(32, len(ws))]
    tnets, _ = make_nets(tws, compute, final_sum, args, "greedy")
    X, t = learned.collect_step_timings(tnets, runs=4)
    model, losses = learned.train_cost_model(X, t, epochs=300, batch=256, lr=2e-3)
    log(f"  {X.shape[0]} step timings, loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    return model


def autotune(nets, args, workload):
    """Applies htn_autotune when asked; returns its choice (or None)."""
    import torch
    from paper_2410_15080_amd import htn
    if args.autotune == "off" or (args.autotune == "auto" and workload not in ("random", "ring")):
        return None
    log("autotuning the fused kernel configuration")
    tmp = torch.empty(len(nets), dtype=torch.float64, device="cuda")
    th, lds, ms = htn.htn_autotune(nets, [tmp[i:i + 1] for i in range(len(nets))])
    log(f"  {th} threads, {lds} B LDS: {ms:.3f} ms")
    return {"threads": th, "lds_bytes": lds, "tuned_ms": round(ms, 4)}


def batch_runner(nets, out_dtype, use_graph=False):
    import torch
    from paper_2410_15080_amd import htn
    dev = torch.device("cuda:0")
    out = torch.empty(len(nets), dtype=out_dtype, device=dev)
    outs = htn.pointer_array([out[i:i + 1] for i in range(len(nets))])
    b = htn.htn_batch_create(nets)
    htn.htn_batch_set_graph(b, use_graph)
    stream = torch.cuda.Stream()
    return b, out, outs, stream


# ------------------------------------------------------------------ grid

def bench_grid(args):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
    n_nets = args.batch or 1024
    args.lds = args.lds or 81920
    log(f"generating {n_nets} grid networks")
    ws = [configs.grid_network(s) for s in range(n_nets)]
    nets, greedy_list = make_nets(ws, htn.HTN_F64, htn.HTN_SUM_PLAIN, args, "greedy")
    greedy_mults = float(sum(greedy_list))
    b, out, outs, stream = batch_runner(nets, torch.float64)
    timer = Timer(stream)
    log("timing the batch on FLOP-greedy paths")
    g_ms, _ = timer.run(lambda: htn.htn_batch_run(b, outs, stream), max(3, args.steps // 2), 2)
    g_res = out.cpu().numpy()
    htn.htn_batch_destroy(b)
    args.path = args.path or "sampled"
    args.samples = args.samples or 128
    if args.path != "greedy":
        log(f"planning {args.path} paths")
        nets, _ = make_nets(ws, htn.HTN_F64, htn.HTN_SUM_PLAIN, args, args.path)
    infos = [htn.htn_get_info(n) for n in nets]
    mults = float(sum(i.mults for i in infos))
    in_bytes = sum(i.input_bytes for i in infos)
    b, out, outs, stream = batch_runner(nets, torch.float64)
    timer = Timer(stream)
    log(f"timing {args.steps} steps")
    ms_per_step, kern_ms = timer.run(lambda: htn.htn_batch_run(b, outs, stream), args.steps, args.warmup,
                                     after_warmup=lambda: htn.htn_batch_set_event_timing(b, True))
    prep_ms, fused_ms, runs = htn.htn_batch_launch_ms(b)
    assert runs == args.steps
    got = out.cpu().numpy()
    eager_ms = ms_per_step
    # the same batch replayed as a captured HIP graph (the timed line; the
    # eager run above gives the per-launch event timing)
    gb, gout, gouts, gstream = batch_runner(nets, torch.float64, use_graph=True)
    log(f"timing {args.steps} graph launches")
    ms_per_step, _ = Timer(gstream).run(lambda: htn.htn_batch_run(gb, gouts, gstream), args.steps, args.warmup)
    assert np.array_equal(gout.cpu().numpy(), got), "graph replay differs from the eager run"
    htn.htn_batch_destroy(gb)
    errs = []
    for i in range(0, n_nets, max(1, n_nets // 32)):
        ref = oracle_ref(ws[i])
        errs.append(max(abs(got[i] - ref), abs(g_res[i] - ref)) / abs(ref))
    htns = n_nets / (ms_per_step * 1e-3)

    plain = None
    if not args.no_plain:
        n_plain = min(n_nets, 256)
        pnets, pm = make_nets(ws[:n_plain], htn.HTN_F64, htn.HTN_SUM_PLAIN, args, "greedy")
        pouts = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in range(n_plain)]
        for n in pnets:
            htn.htn_set_option(n, htn.HTN_OPT_EXEC, htn.HTN_EXEC_STEPS)

        def plain_all():
            for n, o in zip(pnets, pouts):
                htn.htn_contract(n, o, stream)
        log(f"timing plain per-network path on {n_plain} networks")
        p_ms, _ = Timer(stream).run(plain_all, 1, 1)
        pv = np.array([float(o.item()) for o in pouts])
        plain = {"htns_per_s": n_plain / (p_ms * 1e-3), "gflops": 2.0 * sum(pm) / (p_ms * 1e-3) / 1e9,
                 "networks": n_plain, "path": "flop-greedy",
                 "max_abs_diff_vs_batched": float(np.abs(pv - got[:n_plain]).max())}

    cpu = None
    if not args.no_cpu:
        log("timing CPU oracle")
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
    achieved = 2.0 * mults / (fused_ms * 1e-3) / 1e12
    return {
        "metric": METRIC,
        "value": round(2.0 * greedy_mults / (ms_per_step * 1e-3) / 1e9, 3), "unit": "GFLOP/s",
        "ms_per_step": round(ms_per_step, 4), "dtype": "f64",
        "config": {"workload": "grid4x4_htn_batch", "networks": n_nets, "qts_per_net": 16,
                   "cuts_per_net": 24, "cut_dims": "wire 4 / CZ gate 6, 50/50 by seed",
                   "path": args.path, "path_samples": args.samples,
                   "executor": "input prep + fused kernel, one workgroup per network, HIP graph",
                   "lds_budget_bytes": args.lds, "threads_per_network": args.threads,
                   "fused_networks": sum(1 for i in infos if i.fused_ok)},
        "htns_per_s": round(htns, 1),
        "eager_ms_per_step": round(eager_ms, 4),
        "max_rel_err_vs_oracle": float(max(errs)),
        "greedy_mults_per_step": greedy_mults,
        "executed_mults_per_step": mults,
        "batched_greedy_path": {"ms_per_step": round(g_ms, 4), "htns_per_s": round(n_nets / (g_ms * 1e-3), 1),
                                "gflops": round(2.0 * greedy_mults / (g_ms * 1e-3) / 1e9, 3)},
        "plain_fp64_path": plain,
        "speedup_vs_plain_fp64": (htns / plain["htns_per_s"]) if plain else None,
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK["f64_valu"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64_valu"], 5),
                     "traffic": measured_traffic("k_fused_grid", runs_ok=(args.lds == 81920 and args.threads == 256
                                                                           and args.path == "sampled"
                                                                           and args.samples == 128)),
                     "kernel": "k_fused<256,double,double,0>", "kernel_ms": round(fused_ms, 4),
                     "flops_per_launch": 2.0 * mults, "k_fprep_ms": round(prep_ms, 4),
                     "batch_ms_events": round(kern_ms, 4), "input_bytes": in_bytes},
        "cpu_baseline": cpu,
    }


# ------------------------------------------------------------------- qpd

def bench_qpd(args):
    """Grid h-TNs simplified by QPD sampling (Sec. 4.3): every gate-cut CT is
    drawn --qpd-samples times, its undrawn indices are truncated from the
    CT and its QTs.  One step = the truncation gather over the whole batch
    (one launch) + the batch contraction of the simplified networks."""
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
    n_nets = args.batch or 1024
    s_qpd = args.qpd_samples
    args.lds = args.lds or 81920
    args.path = args.path or "sampled"
    args.samples = args.samples or 128
    dev = torch.device("cuda:0")
    log(f"generating {n_nets} grid networks, sampling gate cuts with s_QPD = {s_qpd}")
    ws = [configs.grid_network(s) for s in range(n_nets)]
    rng = np.random.default_rng(2410)
    items, nets, src_keep, sampled = [], [], [], []
    t_sample = 0.0
    for w in ws:
        src = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(dev) for t in w.tensors]
        gate = [i for i, t in enumerate(w.tensors) if w.kinds[i] == "ct" and t.size == 6]
        kept_of, counts, new = {}, {}, list(src)
        for c in gate:
            u = rng.random(s_qpd)
            t0 = time.perf_counter()
            n, wts = htn.htn_qpd_sample(w.tensors[c], s_qpd, u)
            t_sample += time.perf_counter() - t0
            k = np.nonzero(n)[0]
            kept_of[w.labels[c][0]] = k
            counts[c] = n
            new[c] = torch.from_numpy(wts[k]).to(dev)
        dims = list(w.dims)
        for lab, k in kept_of.items():
            dims[lab] = len(k)
        for t, ls in enumerate(w.labels):
            if t in counts or not any(l in kept_of for l in ls):
                continue
            dst = torch.empty(tuple(dims[l] for l in ls), dtype=torch.float64, device=dev)
            items.append((src[t], dst, tuple(w.dims[l] for l in ls), [kept_of.get(l) for l in ls]))
            new[t] = dst
        n = htn.htn_create(new, w.labels, dims, [], compute=htn.HTN_F64)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, args.lds)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_THREADS, args.threads)
        nets.append(n)
        src_keep.append((src, new))
        sampled.append((gate, [counts[c] for c in gate], dims))
    tr = htn.htn_truncate_create(items, htn.HTN_F64)
    trunc_bytes = 2 * 8 * sum(int(np.prod(it[1].shape)) for it in items)
    stream = torch.cuda.Stream()
    htn.htn_truncate_run(tr, stream)
    stream.synchronize()
    greedy_list = [htn.htn_get_info(n).mults for n in nets]
    greedy_mults = float(sum(greedy_list))
    log(f"planning {args.path} paths")
    for n in nets:
        htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, args.samples)
        htn.htn_set_path(n, htn.HTN_PATH_SAMPLED if args.path == "sampled" else htn.HTN_PATH_GREEDY)
    infos = [htn.htn_get_info(n) for n in nets]
    mults = float(sum(i.mults for i in infos))
    b, out, outs, stream = batch_runner(nets, torch.float64)
    timer = Timer(stream)

    def step():
        htn.htn_truncate_run(tr, stream)
        htn.htn_batch_run(b, outs, stream)
    log(f"timing {args.steps} steps")
    ms_per_step, kern_ms = timer.run(step, args.steps, args.warmup,
                                     after_warmup=lambda: htn.htn_batch_set_event_timing(b, True))
    prep_ms, fused_ms, runs = htn.htn_batch_launch_ms(b)
    assert runs == args.steps
    got = out.cpu().numpy()
    log("timing the truncation launch alone")
    _, trunc_ms = Timer(stream).run(lambda: htn.htn_truncate_run(tr, stream), args.steps, args.warmup)
    # parity on a sample of the networks: the oracle's own draws from the
    # same counts, truncation and double-double contraction
    from oracle import qpd_sampling as qs
    errs, ref_ws = [], []
    for i in range(0, n_nets, max(1, n_nets // 32)):
        gate, cnts, dims = sampled[i]
        rw = qs.truncate(ws[i], gate, cnts, s_qpd)
        assert rw.dims == dims
        ref = oracle_ref(rw)
        errs.append(abs(got[i] - ref) / abs(ref))
        ref_ws.append(rw)
    htns = n_nets / (ms_per_step * 1e-3)
    cpu = None
    if not args.no_cpu:
        log("timing CPU oracle")
        cpu = cpu_baseline([qs.truncate(ws[i], *sampled[i][:2], s_qpd) for i in range(min(n_nets, 4096))],
                           args.cpu_seconds, greedy_list)
    achieved = 2.0 * mults / (fused_ms * 1e-3) / 1e12
    tr_gbs = trunc_bytes / (trunc_ms * 1e-3) / 1e9
    htn.htn_truncate_destroy(tr)
    return {
        "metric": METRIC,
        "value": round(2.0 * greedy_mults / (ms_per_step * 1e-3) / 1e9, 3), "unit": "GFLOP/s",
        "ms_per_step": round(ms_per_step, 4), "dtype": "f64",
        "config": {"workload": "grid4x4_htn_batch_qpd_sampled", "networks": n_nets, "qts_per_net": 16,
                   "cuts_per_net": 24, "cut_dims": "wire 4 / CZ gate 6, 50/50 by seed",
                   "qpd_samples_per_gate_ct": s_qpd, "path": args.path, "path_samples": args.samples,
                   "executor": "truncation gather + input prep + fused kernel, one workgroup per network",
                   "lds_budget_bytes": args.lds, "threads_per_network": args.threads},
        "htns_per_s": round(htns, 1),
        "max_rel_err_vs_oracle": float(max(errs)),
        "greedy_mults_per_step": greedy_mults,
        "executed_mults_per_step": mults,
        "host_sampling_ms_per_batch": round(t_sample * 1e3, 3),
        "k_truncate": {"ms": round(trunc_ms, 4), "algorithmic_bytes": trunc_bytes, "items": len(items),
                       "achieved_gbs": round(tr_gbs, 1), "frac_of_hbm_peak": round(tr_gbs / PEAK["hbm_gbs"], 4),
                       "traffic": measured_traffic("k_truncate_qpd8", runs_ok=(s_qpd == 8 and n_nets == 1024))},
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK["f64_valu"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64_valu"], 5), "traffic": None,
                     "kernel": f"k_fused<{args.threads},double,double,0>", "kernel_ms": round(fused_ms, 4),
                     "flops_per_launch": 2.0 * mults, "k_fprep_ms": round(prep_ms, 4),
                     "batch_ms_events": round(kern_ms, 4)},
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------- random

def bench_random(args):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
    n_nets = args.batch or 512
    compute = dtype_code(args.dtype or "f32")
    log(f"generating {n_nets} random networks")
    ws = configs.random_batch(0, n=n_nets, dtype=np.float64)
    args.path = args.path or "learned"
    args.samples = args.samples or 128
    # the fused configuration is tuned first (on FLOP-greedy paths) so that
    # the cost model is trained, and the paths are chosen, under the
    # configuration the batch then runs with
    gnets, greedy_list = make_nets(ws, compute, htn.HTN_SUM_FP64, args, "greedy")
    tuned = autotune(gnets, args, "random")
    del gnets
    if tuned:
        args.threads, args.lds = tuned["threads"], tuned["lds_bytes"]
    nets, _ = make_nets(ws, compute, htn.HTN_SUM_FP64, args, args.path)
    if tuned and args.path != "greedy":
        tuned = autotune(nets, args, "random")  # again, for the chosen paths
    greedy_mults = float(sum(greedy_list))
    infos = [htn.htn_get_info(n) for n in nets]
    mults = float(sum(i.mults for i in infos))
    in_bytes = sum(i.input_bytes for i in infos)

    def path_leg(path):
        """The same batch on other paths (same fused configuration), graph
        launches timed the same way."""
        pn, _ = make_nets(ws, compute, htn.HTN_SUM_FP64, args, path)
        if tuned:
            for n in pn:
                htn.htn_set_option(n, htn.HTN_OPT_FUSED_THREADS, tuned["threads"])
                htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, tuned["lds_bytes"])
        pb, _, pouts, pst = batch_runner(pn, torch.float64, use_graph=True)
        p_ms, _ = Timer(pst).run(lambda: htn.htn_batch_run(pb, pouts, pst), args.steps, args.warmup)
        htn.htn_batch_destroy(pb)
        return {"ms_per_step": round(p_ms, 4), "htns_per_s": round(n_nets / (p_ms * 1e-3), 1),
                "executed_mults_per_step": float(sum(htn.htn_get_info(n).mults for n in pn))}

    legs = {}
    for leg in ("greedy", "sampled"):
        if leg != args.path:
            log(f"timing the batch on {leg} paths")
            legs[leg] = path_leg(leg)
    n_fused = sum(1 for n in nets if json.loads(htn.htn_plan_json(n))["fused_batch_ok"])
    b, out, outs, stream = batch_runner(nets, torch.float64, use_graph=True)
    log(f"timing {args.steps} graph launches")
    ms_per_step, kern_ms = Timer(stream).run(lambda: htn.htn_batch_run(b, outs, stream), args.steps, args.warmup)
    got = out.cpu().numpy()
    t = htn.htn_batch_timestamps(b)
    lat_us = t[:, 1] / 100.0
    # error on every network the oracle finishes quickly
    errs, bounds = [], []
    import oracle
    for i, w in enumerate(ws):
        if greedy_list[i] > 2e6:
            continue
        ref = oracle_ref(w)
        absw = [np.abs(x) for x in w.tensors]
        hi, lo = oracle.ve_contract(absw, w.labels, w.dims, w.out_labels)
        errs.append(abs(got[i] - ref))
        bounds.append(float(hi) + float(lo))
    errs, bounds = np.array(errs), np.array(bounds)
    cpu = None
    if not args.no_cpu:
        log("timing CPU oracle")
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
    achieved = 2.0 * mults / (kern_ms * 1e-3) / 1e12
    peak = PEAK["f32_valu"] if compute != htn.HTN_F64 else PEAK["f64_valu"]
    return {
        "metric": METRIC,
        "value": round(2.0 * greedy_mults / (ms_per_step * 1e-3) / 1e9, 3), "unit": "GFLOP/s",
        "ms_per_step": round(ms_per_step, 4), "dtype": args.dtype or "f32",
        "config": {"workload": "random_htn_batch", "networks": n_nets, "qts": "U{3..12}", "cuts": "U{s-1..14}",
                   "final_sum": "fp64", "path": args.path, "graph": True, "autotuned": tuned,
                   "fused_capable_networks": n_fused},
        "htns_per_s": round(n_nets / (ms_per_step * 1e-3), 1),
        "latency_us": {"p50": float(np.percentile(lat_us, 50)), "p99": float(np.percentile(lat_us, 99)),
                       "max": float(lat_us.max())},
        "error_vs_oracle": {"networks": int(errs.size),
                            "max_abs_err_over_abs_network": float((errs / np.maximum(bounds, 1e-300)).max())},
        "greedy_mults_per_step": greedy_mults, "executed_mults_per_step": mults,
        "other_paths": legs,
        "speedup_vs_flop_greedy": (round(legs["greedy"]["ms_per_step"] / ms_per_step, 3) if "greedy" in legs
                                   else None),
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5), "traffic": None,
                     "kernel": "graph: k_fused + k_fprep + per-step kernels of the largest networks",
                     "kernel_ms": round(kern_ms, 4), "input_bytes": in_bytes,
                     "hbm_gbs_on_inputs": round(in_bytes / (kern_ms * 1e-3) / 1e9, 2)},
        "cpu_baseline": cpu,
    }


# -------------------------------------------------------------- marginal

def bench_marginal(args):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
    import oracle
    name = args.dtype or "f64"
    compute = dtype_code(name)
    w = configs.marginal_network(0, out_bits=12)
    nets, greedy = make_nets([w], compute, htn.HTN_SUM_FP64, args, "greedy")
    net = nets[0]
    htn.htn_set_option(net, htn.HTN_OPT_EXEC, htn.HTN_EXEC_STEPS)
    plan = json.loads(htn.htn_plan_json(net))
    gemm = [s for s in plan["steps"] if s.get("mfma")]
    out = torch.empty(4096 * 4096, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    log("timing the marginal contraction")
    ms, kern_ms = Timer(stream).run(lambda: htn.htn_contract(net, out, stream), args.steps, args.warmup)
    R = out.view(4096, 4096).cpu().numpy()
    # sampled entries against the naive oracle on sliced tensors
    rng = np.random.default_rng(0)
    c = 4
    errs = []
    for _ in range(16):
        x1, x2 = (int(v) for v in rng.integers(0, 4096, size=2))
        ts = [w.tensors[0][..., x1], w.tensors[1][..., x2]] + list(w.tensors[2:])
        ls = [w.labels[0][:c], w.labels[1][:c]] + list(w.labels[2:])
        ref, _ = oracle.naive_contract(ts, ls, w.dims, [])
        errs.append(abs(R[x1, x2] - float(ref)))
    gflop = 2.0 * greedy[0] / 1e9
    mf = 2.0 * float(np.prod(gemm[0]["gemm"])) / 1e9 if gemm else gflop
    peak = {"f64": PEAK["f64_mfma"], "f32": PEAK["f32_mfma"], "bf16": PEAK["bf16_mfma"]}[name]
    achieved = mf / (kern_ms * 1e-3) / 1e3
    out_bytes = 4096 * 4096 * 8
    cpu = None
    if not args.no_cpu:
        # oracle: the naive sum on a block of outputs, scaled per output
        log("timing CPU oracle")
        blk = 8
        ts = [w.tensors[0][..., :blk], w.tensors[1][..., :blk]] + list(w.tensors[2:])
        dims = list(w.dims)
        dims[2 * c] = dims[2 * c + 1] = blk
        t0 = time.perf_counter()
        oracle.naive_contract(ts, w.labels, dims, w.out_labels)
        dt = (time.perf_counter() - t0) * (4096 / blk) ** 2
        cpu = {"value": gflop / dt, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": f"naive knitting sum on an {blk}x{blk} output block, scaled to 4096x4096 "
                         f"(extrapolated: {dt:.0f} s)"}
    return {
        "metric": METRIC,
        "value": round(gflop / (ms * 1e-3), 3), "unit": "GFLOP/s", "ms_per_step": round(ms, 4), "dtype": name,
        "config": {"workload": "marginal_4096x4096", "qts": "2 x [4^4 x 4096]", "cut_tensors": "4 x CutQC c_w",
                   "gemm": gemm[0]["gemm"] if gemm else None, "output": "fp64 4096x4096"},
        "htns_per_s": round(1.0 / (ms * 1e-3), 2),
        "sum_minus_one": float(R.sum() - 1.0),
        "max_abs_err_sampled": float(max(errs)),
        "roofline": {"bound": "mfma" if name != "bf16" else "hbm",
                     "achieved": round(achieved if name != "bf16" else out_bytes / (kern_ms * 1e-3) / 1e9, 3),
                     "peak": peak if name != "bf16" else PEAK["hbm_gbs"],
                     "unit": "TFLOP/s" if name != "bf16" else "GB/s",
                     "frac": round(achieved / peak if name != "bf16" else out_bytes / (kern_ms * 1e-3) / 1e9
                                   / PEAK["hbm_gbs"], 4),
                     "traffic": None, "kernel": "k_gemm (+ pack and fold steps)", "kernel_ms": round(kern_ms, 4)},
        "cpu_baseline": cpu,
    }


# ------------------------------------------------------------------ ring

def bench_ring(args):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
    n_nets = args.batch or 256
    name = args.dtype or "f64"
    compute = dtype_code(name)
    log(f"generating {n_nets} ring-of-rings networks")
    ws = [configs.ring_of_rings(s) for s in range(n_nets)]
    # default FLOP-greedy: planning sampled candidates of 64-QT networks
    # costs ~0.5 s each on the host
    path = args.path or "greedy"
    args.samples = args.samples or 32
    nets, greedy_list = make_nets(ws, compute, htn.HTN_SUM_COMPENSATED, args, path)
    infos = [htn.htn_get_info(n) for n in nets]
    mults = float(sum(i.mults for i in infos))
    in_bytes = sum(i.input_bytes for i in infos)
    tuned = autotune(nets, args, "ring")
    b, out, outs, stream = batch_runner(nets, torch.float64, use_graph=True)
    log(f"timing {args.steps} graph launches")
    ms, kern_ms = Timer(stream).run(lambda: htn.htn_batch_run(b, outs, stream), args.steps, args.warmup)
    got = out.cpu().numpy()
    rel, over_abs = [], []
    import oracle
    for i in range(0, n_nets, max(1, n_nets // 16)):
        ref = oracle_ref(ws[i])
        rel.append(abs(got[i] - ref) / abs(ref))
        # the same error against the contraction of |entries| (the scale the
        # forward error bounds of reduced-precision inputs are stated on)
        hi, lo = oracle.ve_contract([np.abs(x) for x in ws[i].tensors], ws[i].labels, ws[i].dims, ws[i].out_labels)
        over_abs.append(abs(got[i] - ref) / (float(hi) + float(lo)))
    cpu = None
    if not args.no_cpu:
        log("timing CPU oracle")
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
    gbs = in_bytes / (kern_ms * 1e-3) / 1e9
    return {
        "metric": METRIC,
        "value": round(2.0 * float(sum(greedy_list)) / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s",
        "ms_per_step": round(ms, 4), "dtype": name,
        "config": {"workload": "ring_of_rings_batch", "networks": n_nets, "qts_per_net": 64,
                   "final_sum": "compensated fp64", "path": path, "graph": True, "autotuned": tuned},
        "htns_per_s": round(n_nets / (ms * 1e-3), 1),
        "max_rel_err_vs_oracle": float(max(rel)), "median_rel_err_vs_oracle": float(np.median(rel)),
        "max_abs_err_over_abs_network": float(max(over_abs)),
        "greedy_mults_per_step": float(sum(greedy_list)), "executed_mults_per_step": mults,
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                     "frac": round(gbs / PEAK["hbm_gbs"], 5), "traffic": None, "input_bytes": in_bytes,
                     "kernel": "graph: k_fprep + k_fused", "kernel_ms": round(kern_ms, 4)},
        "cpu_baseline": cpu,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (networks of a batch "
              "are independent and would shard across GPUs without communication)", file=sys.stderr)
        return 2
    import torch
    torch.cuda.set_device(0)
    if args.workload not in ("grid", "qpd"):
        args.lds = args.lds or 65536
    fn = {"grid": bench_grid, "random": bench_random, "marginal": bench_marginal, "ring": bench_ring,
          "qpd": bench_qpd}[args.workload]
    line = fn(args)
    head = {"metric": line.pop("metric"), "value": line.pop("value"), "unit": line.pop("unit"), "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": line.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": line.pop("dtype"),
            "data": "synthetic", "config": line.pop("config")}
    head.update(line)
    print(json.dumps(head), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
