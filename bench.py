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
  qpd        the grid batch after QPD sampling of every gate cut (truncation
             gather + contraction of the simplified networks)
  copy-calibration  a plain 64 MiB device copy, the reference run that
             scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes

With the default grid workload (and --configs all) the line also carries
"configs": every other workload (the 10-qubit circuit's latency, the
marginal in FP64/FP32/BF16, the ring batch in FP64/FP32/BF16, the random
serving batch on learned paths, the QPD-sampled grid) in the same form,
with fewer timed steps and a shorter CPU sample each.

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
    ap.add_argument("--workload", choices=["grid", "random", "marginal", "ring", "qpd", "copy-calibration"],
                    default="grid")
    ap.add_argument("--configs", choices=["all", "none"], default="all",
                    help="with the grid workload: also run every other workload and nest its results "
                         "under \"configs\" (all, the default) or not (none)")
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
    ap.add_argument("--queue", choices=["auto", "all", "off"], default="auto",
                    help="batch work queue: networks run step by step go to it (auto), every network "
                         "does (all), or each step is its own launch (off)")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="measure the fused kernel's workgroup size and LDS budget first "
                         "(auto: on for the random and ring batches)")
    return ap.parse_args()


# HBM traffic per launch of a kernel on a workload, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this script scaled by the same counters
# on a plain copy (profiles/ holds the summaries and commands).  Each record
# carries a digest of the sources that shape the kernel and its plans; when
# they change the record no longer applies and traffic is reported as null.
MARGINAL_TRAFFIC_FILES = ["paper_2410_15080_amd/csrc/" + f for f in (
    "mfma.hip", "mfma_dev.hpp", "kernels.hip", "kernels.hpp", "step_dev.hpp", "kern_common.hpp", "planner.cpp", "api.hip")]
TRAFFIC = {
    # profiles/k_fused_grid4x4_batch1024_f64.md: FETCH_SIZE 18 716.2 x 2047.2 B, WRITE_SIZE 181.1 x 1024 B
    "k_fused_grid": {"read_bytes": 38_315_694, "write_bytes": 185_446, "sources": "b23f60e326e35d2a",
                     "profile": "profiles/k_fused_grid4x4_batch1024_f64.md"},
    # profiles/k_truncate_grid4x4_qpd8_batch1024_f64.md: FETCH_SIZE 13 479.3 x 2047.2 B, WRITE_SIZE 15 553.6 x 1024 B
    "k_truncate_qpd8": {"read_bytes": 27_594_743, "write_bytes": 15_926_886, "sources": "e5762072f8252300",
                        "files": ["paper_2410_15080_amd/csrc/qpd.hip", "paper_2410_15080_amd/csrc/api.hip",
                                  "paper_2410_15080_amd/csrc/kernels.hpp"],
                        "profile": "profiles/k_truncate_grid4x4_qpd8_batch1024_f64.md"},
    # profiles/k_gemm_marginal4096_f64_f32_bf16.md: one contraction's kernels
    # (k_fold, k_gemm), FETCH_SIZE x 2047.2 B and WRITE_SIZE x 1024 B summed
    "marginal_bf16": {"read_bytes": 23_626_944, "write_bytes": 138_531_328, "sources": "fc6d7fa7bfcade02",
                      "files": MARGINAL_TRAFFIC_FILES, "profile": "profiles/k_gemm_marginal4096_f64_f32_bf16.md"},
    "marginal_f64": {"read_bytes": 99_749_016, "write_bytes": 151_014_810, "sources": "fc6d7fa7bfcade02",
                     "files": MARGINAL_TRAFFIC_FILES, "profile": "profiles/k_gemm_marginal4096_f64_f32_bf16.md"},
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ws, seconds, mults):
    """Time the oracle (FP64 variable elimination) on every host core in the
    affinity mask, one network per thread: a warm-up pass, then the best of
    three passes over a sample sized so that one pass takes about seconds/4."""
    import oracle
    cores = max(1, len(os.sched_getaffinity(0)))
    oracle.set_num_threads(1)

    def one(w):
        return oracle.ve_contract(w.tensors, w.labels, w.dims, w.out_labels, mode="f64")

    with concurrent.futures.ThreadPoolExecutor(max_workers=cores) as ex:
        # size the sample: grow it until one pass takes seconds / 4
        budget = max(0.5, seconds / 4.0)
        n = min(len(ws), cores)
        while True:
            t0 = time.perf_counter()
            list(ex.map(one, ws[:n]))
            dt = time.perf_counter() - t0
            if n >= len(ws) or dt >= budget:
                break
            n = min(len(ws), max(n + cores, int(n * min(8.0, 1.2 * budget / max(dt, 1e-3)))))
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            list(ex.map(one, ws[:n]))
            best = min(best, time.perf_counter() - t0)
    oracle.set_num_threads(cores)
    cm = float(sum(mults[:n]))
    return {"value": 2.0 * cm / best / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "htns_per_s": n / best, "cpu_model": cpu_model(),
            "sample": f"first {n} of the {len(ws)} networks, FP64 variable elimination, one network per "
                      f"thread on {cores} threads, best of 3 passes after a warm-up ({best:.2f} s per pass)"}


def roofline(flops, nbytes, seconds, flop_peak_tf, unit_peak_name, **extra):
    """Both roofline fractions of a kernel from its algorithmic flops and HBM
    bytes per launch and its launch duration; the bound is the unit the
    arithmetic intensity points at (flops / bytes against the ridge
    peak_flops / peak_bandwidth), and the reported fraction is that unit's."""
    fps = flops / seconds / 1e12
    bps = nbytes / seconds / 1e9
    ridge = flop_peak_tf * 1e12 / (PEAK["hbm_gbs"] * 1e9)
    intensity = flops / nbytes if nbytes else float("inf")
    f_frac = fps / flop_peak_tf
    b_frac = bps / PEAK["hbm_gbs"]
    if intensity < ridge:
        r = {"bound": "hbm", "achieved": round(bps, 2), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
             "frac": round(b_frac, 5)}
    else:
        r = {"bound": unit_peak_name, "achieved": round(fps, 4), "peak": flop_peak_tf, "unit": "TFLOP/s",
             "frac": round(f_frac, 5)}
    r.update({"intensity_flop_per_byte": round(intensity, 3), "ridge_flop_per_byte": round(ridge, 3),
              "flop_frac": round(f_frac, 5), "hbm_frac": round(b_frac, 5), "algorithmic_flops": flops,
              "algorithmic_bytes": nbytes})
    r.update(extra)
    return r


# The CPU leg of each workload (skipped with --no-cpu) is the only part of
# this script that runs the oracle: it times the oracle on the host cores
# (cpu_baseline) and checks the GPU results against it (the *_vs_oracle
# figures).


def oracle_ref(w):
    """CPU leg: the oracle's double-double value of a network."""
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
        htn.htn_set_option(n, htn.HTN_OPT_QUEUE, {"auto": 0, "all": 1, "off": 2}[args.queue])
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
        p_ms = median_wall_ms(plain_all, stream, reps=7, warmup=1)
        pv = np.array([float(o.item()) for o in pouts])
        plain = {"htns_per_s": n_plain / (p_ms * 1e-3), "gflops": 2.0 * sum(pm) / (p_ms * 1e-3) / 1e9,
                 "networks": n_plain, "path": "flop-greedy", "timing": "median of 7 passes after a warm-up",
                 "ms_per_pass": round(p_ms, 3),
                 "max_abs_diff_vs_batched": float(np.abs(pv - got[:n_plain]).max())}

    log("timing one network alone (latency)")
    single = single_latency(ws[0], args)
    cpu, err = None, None
    if not args.no_cpu:
        log("CPU leg: checking against and timing the oracle")
        errs = []
        for i in range(0, n_nets, max(1, n_nets // 32)):
            ref = oracle_ref(ws[i])
            errs.append(max(abs(got[i] - ref), abs(g_res[i] - ref)) / abs(ref))
        err = float(max(errs))
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
    traffic = measured_traffic("k_fused_grid", runs_ok=(args.lds == 81920 and args.threads == 256
                                                       and args.path == "sampled" and args.samples == 128))
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
        "max_rel_err_vs_oracle": err,
        "greedy_mults_per_step": greedy_mults,
        "executed_mults_per_step": mults,
        "batched_greedy_path": {"ms_per_step": round(g_ms, 4), "htns_per_s": round(n_nets / (g_ms * 1e-3), 1),
                                "gflops": round(2.0 * greedy_mults / (g_ms * 1e-3) / 1e9, 3)},
        "plain_fp64_path": plain,
        "speedup_vs_plain_fp64": (htns / plain["htns_per_s"]) if plain else None,
        "single_network": single,
        # k_fused: executed flops of the sampled paths; algorithmic bytes =
        # the batch's inputs read once plus one FP64 result per network
        "roofline": roofline(2.0 * mults, in_bytes + 8 * n_nets, fused_ms * 1e-3, PEAK["f64_valu"], "alu",
                             traffic=traffic, kernel="k_fused<256,double,double,0>", kernel_ms=round(fused_ms, 4),
                             k_fprep_ms=round(prep_ms, 4), batch_ms_events=round(kern_ms, 4),
                             input_bytes=in_bytes),
        "cpu_baseline": cpu,
    }


def median_wall_ms(fn, stream, reps=7, warmup=1):
    """Median wall time of `reps` calls of fn, each bracketed by stream
    synchronisation (for host-bound launch sequences)."""
    import numpy as np
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            fn()
    stream.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            fn()
        stream.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def single_latency(w, args, reps=50):
    """One grid network contracted on its own (htn_contract, fused executor,
    sampled path): median HIP-event latency of `reps` calls after a warm-up,
    and the same through the per-step executor on the FLOP-greedy path."""
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    dev = torch.device("cuda:0")
    ts = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(dev) for t in w.tensors]
    out = torch.empty(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    res = {}
    for name, exec_mode, path in (("fused_sampled", htn.HTN_EXEC_FUSED, htn.HTN_PATH_SAMPLED),
                                  ("steps_greedy", htn.HTN_EXEC_STEPS, htn.HTN_PATH_GREEDY)):
        n = htn.htn_create(ts, w.labels, w.dims, w.out_labels)
        htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, 128)
        htn.htn_set_path(n, path)
        htn.htn_set_option(n, htn.HTN_OPT_EXEC, exec_mode)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        with torch.cuda.stream(stream):
            for _ in range(5):
                htn.htn_contract(n, out, stream)
            stream.synchronize()
            for a, b in ev:
                a.record(stream)
                htn.htn_contract(n, out, stream)
                b.record(stream)
        stream.synchronize()
        res[name + "_us"] = round(1e3 * float(np.median([a.elapsed_time(b) for a, b in ev])), 2)
    res["timing"] = f"median of {reps} HIP-event intervals on the launch stream"
    return res


# ------------------------------------------------------------------- qpd

def bench_qpd(args):
    """Grid h-TNs simplified by QPD sampling (Sec. 4.3): the gate-cut CTs
    between the same QTs are fused (none on a grid: one cut per edge), each
    CT is drawn --qpd-samples times, undrawn indices are truncated from the
    CT and its QTs.  One step = the gather over the whole batch (one
    launch) + the batch contraction of the simplified networks."""
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
    from paper_2410_15080_amd import qpd as lq
    ws = [configs.grid_network(s) for s in range(n_nets)]
    rng = np.random.default_rng(2410)
    items, nets, src_keep, sampled = [], [], [], []
    t_sample = 0.0
    for w in ws:
        src = [torch.from_numpy(np.ascontiguousarray(t, dtype=np.float64)).to(dev) for t in w.tensors]
        gate = [i for i, t in enumerate(w.tensors) if w.kinds[i] == "ct" and t.size == 6]
        uniforms = [rng.random(s_qpd) for _ in lq.parallel_groups(w.labels, gate)]
        t0 = time.perf_counter()
        simp = lq.simplify(src, w.labels, w.dims, w.out_labels, gate, s_qpd, uniforms, items, device=dev)
        t_sample += time.perf_counter() - t0
        n = htn.htn_create(simp.tensors, simp.labels, simp.dims, simp.out_labels, compute=htn.HTN_F64)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, args.lds)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_THREADS, args.threads)
        nets.append(n)
        src_keep.append((src, simp))
        sampled.append((gate, uniforms, simp.dims))
    tr = htn.htn_gather_create(items, htn.HTN_F64)
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
    in_bytes = sum(i.input_bytes for i in infos)
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
    htns = n_nets / (ms_per_step * 1e-3)
    cpu, err = None, None
    if not args.no_cpu:
        # CPU leg: the oracle's own fusion, draws from the same uniforms,
        # truncation and double-double contraction on a sample of the
        # networks, then the oracle timed on the simplified networks
        log("CPU leg: checking against and timing the oracle")
        from oracle import qpd_sampling as qs
        errs = []
        for i in range(0, n_nets, max(1, n_nets // 32)):
            gate, uniforms, dims = sampled[i]
            rw = qs.simplify(ws[i], gate, s_qpd, uniforms)[0]
            assert rw.dims == dims
            ref = oracle_ref(rw)
            errs.append(abs(got[i] - ref) / abs(ref))
        err = float(max(errs))
        cpu = cpu_baseline([qs.simplify(ws[i], sampled[i][0], s_qpd, sampled[i][1])[0] for i in range(n_nets)],
                           args.cpu_seconds, greedy_list)
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
        "max_rel_err_vs_oracle": err,
        "greedy_mults_per_step": greedy_mults,
        "executed_mults_per_step": mults,
        "host_sampling_ms_per_batch": round(t_sample * 1e3, 3),
        "k_truncate": {"ms": round(trunc_ms, 4), "algorithmic_bytes": trunc_bytes, "items": len(items),
                       "achieved_gbs": round(tr_gbs, 1), "frac_of_hbm_peak": round(tr_gbs / PEAK["hbm_gbs"], 4),
                       "traffic": measured_traffic("k_truncate_qpd8", runs_ok=(s_qpd == 8 and n_nets == 1024))},
        "roofline": roofline(2.0 * mults, in_bytes + 8 * n_nets, fused_ms * 1e-3, PEAK["f64_valu"], "alu",
                             traffic=None, kernel=f"k_fused<{args.threads},double,double,0>",
                             kernel_ms=round(fused_ms, 4), k_fprep_ms=round(prep_ms, 4),
                             batch_ms_events=round(kern_ms, 4)),
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
    cpu, err = None, None
    if not args.no_cpu:
        # CPU leg: error on every network the oracle finishes quickly, then
        # the oracle timed
        log("CPU leg: checking against and timing the oracle")
        import oracle
        errs, bounds = [], []
        for i, w in enumerate(ws):
            if greedy_list[i] > 2e6:
                continue
            ref = oracle_ref(w)
            absw = [np.abs(x) for x in w.tensors]
            hi, lo = oracle.ve_contract(absw, w.labels, w.dims, w.out_labels)
            errs.append(abs(got[i] - ref))
            bounds.append(float(hi) + float(lo))
        errs, bounds = np.array(errs), np.array(bounds)
        err = {"networks": int(errs.size),
               "max_abs_err_over_abs_network": float((errs / np.maximum(bounds, 1e-300)).max())}
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
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
        "error_vs_oracle": err,
        "greedy_mults_per_step": greedy_mults, "executed_mults_per_step": mults,
        "other_paths": legs,
        "speedup_vs_flop_greedy": (round(legs["greedy"]["ms_per_step"] / ms_per_step, 3) if "greedy" in legs
                                   else None),
        "roofline": roofline(2.0 * mults, in_bytes + 8 * n_nets, kern_ms * 1e-3, peak, "alu", traffic=None,
                             kernel="graph: k_fprep + k_fused + k_queue / per-step kernels of the largest networks",
                             kernel_ms=round(kern_ms, 4), input_bytes=in_bytes),
        "cpu_baseline": cpu,
    }


# -------------------------------------------------------------- marginal

def bench_marginal(args):
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn
    from workloads import configs
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
    c = 4
    gflop = 2.0 * greedy[0] / 1e9
    mf = 2.0 * float(np.prod(gemm[0]["gemm"])) / 1e9 if gemm else gflop
    peak = {"f64": PEAK["f64_mfma"], "f32": PEAK["f32_mfma"], "bf16": PEAK["bf16_mfma"]}[name]
    out_bytes = 4096 * 4096 * 8
    in_bytes = htn.htn_get_info(net).input_bytes
    cpu, err = None, None
    if not args.no_cpu:
        # CPU leg: sampled entries against the naive oracle on sliced
        # tensors; then the oracle (FP64 variable elimination) timed on whole
        # rows R[x1, :], each row the network with x1 fixed, scaled from the
        # rows timed to all
        log("CPU leg: checking against and timing the oracle")
        import oracle
        rng = np.random.default_rng(0)
        errs = []
        for _ in range(16):
            x1, x2 = (int(v) for v in rng.integers(0, 4096, size=2))
            ts = [w.tensors[0][..., x1], w.tensors[1][..., x2]] + list(w.tensors[2:])
            ls = [w.labels[0][:c], w.labels[1][:c]] + list(w.labels[2:])
            ref, _ = oracle.naive_contract(ts, ls, w.dims, [])
            errs.append(abs(R[x1, x2] - float(ref)))
        err = float(max(errs))
        from workloads.network import Network
        rows = []
        for x1 in range(4096):
            ts = [w.tensors[0][..., x1], w.tensors[1]] + list(w.tensors[2:])
            ls = [w.labels[0][:c], w.labels[1]] + list(w.labels[2:])
            rows.append(Network(ts, ls, w.dims, [w.labels[1][c]], w.kinds, {}))
        cpu = cpu_baseline(rows, args.cpu_seconds, [greedy[0] / 4096.0] * 4096)
        cpu["htns_per_s"] = cpu["htns_per_s"] / 4096.0
        cpu["sample"] = "rows of the marginal (one network per row, x1 fixed): " + cpu["sample"]
    return {
        "metric": METRIC,
        "value": round(gflop / (ms * 1e-3), 3), "unit": "GFLOP/s", "ms_per_step": round(ms, 4), "dtype": name,
        "config": {"workload": "marginal_4096x4096", "qts": "2 x [4^4 x 4096]", "cut_tensors": "4 x CutQC c_w",
                   "gemm": gemm[0]["gemm"] if gemm else None, "output": "fp64 4096x4096"},
        "htns_per_s": round(1.0 / (ms * 1e-3), 2),
        "sum_minus_one": float(R.sum() - 1.0),
        "max_abs_err_sampled": err,
        # the whole contraction (coefficient fold, packs and the GEMM) timed as
        # one: the GEMM's flops over the inputs read once and the FP64
        # result written once
        "roofline": roofline(mf * 1e9, in_bytes + out_bytes, kern_ms * 1e-3, peak, "mfma",
                             traffic=measured_traffic("marginal_" + name) if name != "f32" else None,
                             kernel="whole contraction: fold + pack + k_gemm", kernel_ms=round(kern_ms, 4)),
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
    cpu, errs = None, {"max_rel_err_vs_oracle": None, "median_rel_err_vs_oracle": None,
                       "max_abs_err_over_abs_network": None}
    if not args.no_cpu:
        # CPU leg: the oracle on a sample of the networks, then timed
        log("CPU leg: checking against and timing the oracle")
        import oracle
        rel, over_abs = [], []
        for i in range(0, n_nets, max(1, n_nets // 16)):
            ref = oracle_ref(ws[i])
            rel.append(abs(got[i] - ref) / abs(ref))
            # the same error against the contraction of |entries| (the scale
            # the forward error bounds of reduced-precision inputs are stated on)
            hi, lo = oracle.ve_contract([np.abs(x) for x in ws[i].tensors], ws[i].labels, ws[i].dims,
                                        ws[i].out_labels)
            over_abs.append(abs(got[i] - ref) / (float(hi) + float(lo)))
        errs = {"max_rel_err_vs_oracle": float(max(rel)), "median_rel_err_vs_oracle": float(np.median(rel)),
                "max_abs_err_over_abs_network": float(max(over_abs))}
        cpu = cpu_baseline(ws, args.cpu_seconds, greedy_list)
    peak = PEAK["f64_valu"] if compute == htn.HTN_F64 else PEAK["f32_valu"]
    return {
        "metric": METRIC,
        "value": round(2.0 * float(sum(greedy_list)) / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s",
        "ms_per_step": round(ms, 4), "dtype": name,
        "config": {"workload": "ring_of_rings_batch", "networks": n_nets, "qts_per_net": 64,
                   "final_sum": "compensated fp64", "path": path, "graph": True, "autotuned": tuned},
        "htns_per_s": round(n_nets / (ms * 1e-3), 1),
        **errs,
        "greedy_mults_per_step": float(sum(greedy_list)), "executed_mults_per_step": mults,
        "roofline": roofline(2.0 * mults, in_bytes + 8 * n_nets, kern_ms * 1e-3, peak, "alu", traffic=None,
                             kernel="graph: k_fprep + k_fused + k_queue (networks of many small steps) + per-step kernels", kernel_ms=round(kern_ms, 4),
                             input_bytes=in_bytes),
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------- circuit

def bench_circuit(args):
    """The 10-qubit circuit cut by two wire cuts into three subcircuits, end
    to end on the GPU: the QT evaluator simulates the 44 subcircuit
    instances (one launch) and assembles the QTs [4], [4, 4], [4] (one
    launch), then the library contracts the network.  Latency of the whole
    and of the contraction alone (both executors); the CPU leg checks the
    value against the uncut circuit's statevector and times the oracle
    (statevector QTs plus the naive knitting sum)."""
    import numpy as np
    import torch
    from paper_2410_15080_amd import htn, qteval
    from workloads import circuits
    cn = circuits.cut_wires(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ts, ev = qteval.network_tensors(cn, stream)
    stream.synchronize()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    res = {}
    for name, mode in (("fused", htn.HTN_EXEC_FUSED), ("steps", htn.HTN_EXEC_STEPS)):
        n = htn.htn_create(ts, cn.labels, cn.dims, cn.out_labels)
        htn.htn_set_option(n, htn.HTN_OPT_EXEC, mode)
        for label, fn in (("contract", lambda: htn.htn_contract(n, out, stream)),
                          ("evaluate_and_contract", lambda: (ev.run(stream), htn.htn_contract(n, out, stream)))):
            ev_pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                        for _ in range(50)]
            with torch.cuda.stream(stream):
                for _ in range(5):
                    fn()
                for e0, e1 in ev_pairs:
                    e0.record(stream)
                    fn()
                    e1.record(stream)
            stream.synchronize()
            res[f"{name}_{label}_us"] = round(1e3 * float(np.median([e0.elapsed_time(e1) for e0, e1 in ev_pairs])), 2)
        res[f"{name}_value"] = float(out.item())
    line = {"workload": "circuit10_two_wire_cuts", "qts": "[4], [4,4], [4] from 44 instances (5/4/3 qubits)",
            "latency": res, "timing": "median of 50 HIP-event intervals", "abs_err_vs_statevector": None,
            "cpu_baseline": None}
    if not args.no_cpu:
        # CPU leg: the uncut circuit's statevector, and the oracle timed end to
        # end (statevector QTs, then the naive knitting sum)
        import oracle
        from oracle import statevector as sv
        full = float(sv.full_value(cn))
        line["abs_err_vs_statevector"] = max(abs(res["fused_value"] - full), abs(res["steps_value"] - full))
        t0 = time.perf_counter()
        for _ in range(20):
            w = sv.network(cn)
            oracle.naive_contract(w.tensors, w.labels, w.dims, w.out_labels)
        us = (time.perf_counter() - t0) / 20 * 1e6
        line["cpu_baseline"] = {"value": round(us, 1), "unit": "us per network", "cores": 1, "kind": "oracle",
                                "sample": "statevector QTs (44 instances) + naive knitting sum, mean of 20"}
    return line


def copy_calibration(args):
    """Plain device-to-device copy of 64 MiB, three launches: the reference
    run for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes
    (bytes per counter unit = bytes copied / counter reading)."""
    import torch
    n = 64 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {n * 8} bytes per launch, 3 launches")
    return None


def sub_args(args, **kw):
    """Arguments of a nested configuration run: the defaults of its own
    workload, fewer timed steps, a shorter CPU sample."""
    a = argparse.Namespace(**vars(args))
    a.batch = None
    a.lds = None
    a.threads = 256
    a.path = None
    a.samples = None
    a.dtype = None
    a.autotune = "auto"
    a.steps = max(5, min(args.steps, 10))
    a.warmup = max(2, min(args.warmup, 3))
    a.cpu_seconds = min(args.cpu_seconds, 6.0)
    a.no_plain = True
    for k, v in kw.items():
        setattr(a, k, v)
    if a.workload not in ("grid", "qpd"):
        a.lds = a.lds or 65536
    return a


NESTED = (("circuit10", "circuit", {}),
          ("marginal_f64", "marginal", {"dtype": "f64"}),
          ("marginal_f32", "marginal", {"dtype": "f32"}),
          ("marginal_bf16", "marginal", {"dtype": "bf16"}),
          ("ring_f64", "ring", {"dtype": "f64"}),
          ("ring_f32", "ring", {"dtype": "f32"}),
          ("ring_bf16", "ring", {"dtype": "bf16"}),
          ("random_f32_learned", "random", {"dtype": "f32"}),
          ("qpd_grid_s8", "qpd", {}))


def run_nested(args):
    """Every other workload, each in the same form as its own line, nested
    under the headline line's "configs"."""
    fns = {"circuit": bench_circuit, "random": bench_random, "marginal": bench_marginal, "ring": bench_ring,
           "qpd": bench_qpd}
    out = {}
    for key, wl, kw in NESTED:
        log(f"--- nested configuration {key}")
        t0 = time.perf_counter()
        a = sub_args(args, workload=wl, **kw)
        r = fns[wl](a)
        r.pop("metric", None)
        r["steps"], r["warmup"] = a.steps, a.warmup
        r["run_s"] = round(time.perf_counter() - t0, 1)
        out[key] = r
    return out


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
    if args.workload == "copy-calibration":
        copy_calibration(args)
        return 0
    fn = {"grid": bench_grid, "random": bench_random, "marginal": bench_marginal, "ring": bench_ring,
          "qpd": bench_qpd}[args.workload]
    line = fn(args)
    if args.workload == "grid" and args.configs == "all":
        line["configs"] = run_nested(args)
    head = {"metric": line.pop("metric"), "value": line.pop("value"), "unit": line.pop("unit"), "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": line.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": line.pop("dtype"),
            "data": "synthetic", "config": line.pop("config")}
    head.update(line)
    print(json.dumps(head), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
