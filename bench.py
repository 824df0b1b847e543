#!/usr/bin/env python3
"""h-TN contraction throughput on one MI355X.

Workload (one "step"): a batch of 1024 seeded 4x4-grid h-TNs -- 16 quantum
tensors, 24 cuts, each cut a wire cut (dim 4, Pauli-basis weights 1/2) or a
CZ gate cut (dim 6, six QPD weights) drawn 50/50 per edge, QT entries
U[-1,1] -- contracted in FP64 to each network's scalar <O>.  The batch
runs as one input-materialisation launch plus one launch of the fused
kernel (one workgroup per network).  Inputs are resident in HBM before
timing.

Reported:
  value        GFLOP/s = 2 * (multiplications of the FLOP-greedy paths) / time;
               the same numerator for every path variant, so a cheaper
               path shows up as higher throughput, never as extra flops
  htns_per_s   networks per second
  path         order executed: "sampled" (cheapest of FLOP-greedy and 32
               Boltzmann-sampled greedy paths) by default
  batched_greedy_path  the same batch executed on the FLOP-greedy paths
  plain_fp64   the same networks contracted one at a time on their
               FLOP-greedy paths, one kernel launch per pairwise step
  roofline     the fused kernel against the FP64 vector-ALU peak, on the
               multiplications it actually executes
  cpu_baseline the CPU oracle (FP64 variable elimination) on a bounded
               sample of the same networks, on the host's cores
"""

import argparse
import concurrent.futures
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lds", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--path", choices=["greedy", "sampled", "learned"], default="sampled")
    ap.add_argument("--samples", type=int, default=32)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(ws, seconds):
    """Time the oracle (FP64 variable elimination) on as many networks as fit
    in about `seconds`, one network per host thread."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    cores = max(1, min(cores, 16))
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
    return done, dt, cores


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (networks of a batch "
              "are independent and would shard across GPUs without communication)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import oracle
    from paper_2410_15080_amd import htn
    from workloads import configs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    log(f"generating {args.batch} grid networks")
    ws = [configs.grid_network(s) for s in range(args.batch)]
    nets = []
    greedy_list = []
    for w in ws:
        ts = [torch.from_numpy(np.ascontiguousarray(t)).to(dev) for t in w.tensors]
        n = htn.htn_create(ts, w.labels, w.dims, w.out_labels, compute=htn.HTN_F64)
        htn.htn_set_option(n, htn.HTN_OPT_FUSED_LDS_BYTES, args.lds)
        greedy_list.append(htn.htn_get_info(n).mults)
        nets.append(n)
    greedy_mults = float(sum(greedy_list))
    out = torch.empty(args.batch, dtype=torch.float64, device=dev)
    outs = htn.pointer_array([out[i:i + 1] for i in range(args.batch)])
    stream = torch.cuda.Stream()

    def time_batch(steps, warmup):
        batch = htn.htn_batch_create(nets)
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                htn.htn_batch_run(batch, outs, stream)
        stream.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for k in range(steps):
                ev[k][0].record(stream)
                htn.htn_batch_run(batch, outs, stream)
                ev[k][1].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall * 1e3 / steps, float(np.mean([a.elapsed_time(b) for a, b in ev]))

    # the FLOP-greedy paths (transparency)
    log("timing the batch on FLOP-greedy paths")
    g_ms, _ = time_batch(max(3, args.steps // 2), 2)
    g_res = out.cpu().numpy()
    # the executed path
    if args.path != "greedy":
        log(f"planning {args.path} paths")
        for n in nets:
            htn.htn_set_option(n, htn.HTN_OPT_PATH_SAMPLES, args.samples)
            htn.htn_set_path(n, htn.HTN_PATH_SAMPLED if args.path == "sampled" else htn.HTN_PATH_LEARNED)
    infos = [htn.htn_get_info(n) for n in nets]
    mults = float(sum(i.mults for i in infos))
    n_fused = sum(1 for i in infos if i.fused_ok)
    in_bytes = sum(i.input_bytes for i in infos)
    log(f"timing {args.steps} steps")
    ms_per_step, kern_ms = time_batch(args.steps, args.warmup)
    got = out.cpu().numpy()
    # correctness on a sample against the oracle (double-double)
    errs = []
    for i in range(0, args.batch, max(1, args.batch // 32)):
        hi, lo = oracle.ve_contract(ws[i].tensors, ws[i].labels, ws[i].dims, ws[i].out_labels)
        ref = float(hi) + float(lo)
        errs.append(max(abs(got[i] - ref), abs(g_res[i] - ref)) / abs(ref))
    max_rel = float(max(errs))
    gflops = 2.0 * greedy_mults / (ms_per_step * 1e-3) / 1e9
    htns = args.batch / (ms_per_step * 1e-3)

    plain = None
    if not args.no_plain:
        n_plain = min(args.batch, 256)
        pouts = [torch.empty(1, dtype=torch.float64, device=dev) for _ in range(n_plain)]
        for n in nets[:n_plain]:
            htn.htn_set_path(n, htn.HTN_PATH_GREEDY)
            htn.htn_set_option(n, htn.HTN_OPT_EXEC, htn.HTN_EXEC_STEPS)
        plain_mults = float(sum(htn.htn_get_info(n).mults for n in nets[:n_plain]))
        with torch.cuda.stream(stream):
            for n, o in zip(nets[:n_plain], pouts):
                htn.htn_contract(n, o, stream)
        stream.synchronize()
        log(f"timing plain per-network path on {n_plain} networks")
        t1 = time.perf_counter()
        with torch.cuda.stream(stream):
            for n, o in zip(nets[:n_plain], pouts):
                htn.htn_contract(n, o, stream)
        stream.synchronize()
        dtp = time.perf_counter() - t1
        pm = float(sum(i.mults for i in infos[:n_plain]))
        pv = np.array([float(o.item()) for o in pouts])
        plain = {"htns_per_s": n_plain / dtp, "gflops": 2.0 * plain_mults / dtp / 1e9, "networks": n_plain,
                 "path": "flop-greedy",
                 "max_abs_diff_vs_batched": float(np.abs(pv - got[:n_plain]).max())}

    cpu = None
    if not args.no_cpu:
        log("timing CPU oracle")
        done, dtc, cores = cpu_baseline(ws, args.cpu_seconds)
        cm = float(sum(greedy_list[:done]))  # same numerator as the headline
        cpu = {"value": 2.0 * cm / dtc / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
               "htns_per_s": done / dtc,
               "sample": f"first {done} of the {args.batch} grid networks, FP64 variable elimination, "
                         f"one network per thread, {dtc:.1f} s"}

    achieved = 2.0 * mults / (kern_ms * 1e-3) / 1e12
    greedy_batched = {"ms_per_step": round(g_ms, 4), "htns_per_s": round(args.batch / (g_ms * 1e-3), 1),
                      "gflops": round(2.0 * greedy_mults / (g_ms * 1e-3) / 1e9, 3)}
    line = {
        "metric": "h-TN contraction GFLOP/s & h-TNs/s vs plain FP64 path, at stated rel. error",
        "value": round(gflops, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "grid4x4_htn_batch", "networks": args.batch, "qts_per_net": 16,
                   "cuts_per_net": 24, "cut_dims": "wire 4 / CZ gate 6, 50/50 by seed",
                   "path": args.path, "path_samples": args.samples,
                   "executor": "input prep + fused kernel, one workgroup per network",
                   "lds_budget_bytes": args.lds, "fused_networks": n_fused},
        "htns_per_s": round(htns, 1),
        "max_rel_err_vs_oracle": max_rel,
        "greedy_mults_per_step": greedy_mults,
        "executed_mults_per_step": mults,
        "batched_greedy_path": greedy_batched,
        "plain_fp64_path": plain,
        "speedup_vs_plain_fp64": (htns / plain["htns_per_s"]) if plain else None,
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 5), "traffic": None,
                     "kernel": "k_fused<double,double>", "kernel_ms": round(kern_ms, 4),
                     "input_bytes": in_bytes},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
