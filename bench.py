#!/usr/bin/env python3
"""Benchmark: multiplicative-update sweeps per second on one MI355X.

Workload (default): CP model 'ir,jr,kr->ijk', 256 x 256 x 256, rank 32, Poisson
counts from Gamma(0.3, 1) factors, 20 % of entries missing, (alpha, beta) =
(1, 1) in the paper's convention, plain FP32 contractions.  A step is one sweep
of Algorithm 1 (three block updates).  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line with the sweep rate, the roofline of the dominant kernel
(the fused pass over Y) measured live with HIP events on the stream it runs on,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}  # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0  # GB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--beta", type=float, default=1.0)
    ap.add_argument("--n", type=int, default=256, help="mode size")
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--prec", choices=("fp32", "bf16", "fp16"), default="fp32",
                    help="input precision of the N/D contractions")
    ap.add_argument("--cpu-sweeps", type=int, default=3,
                    help="oracle sweeps timed for the CPU baseline (0 disables)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of Y (a reference for HBM counters)")
    return ap.parse_args()


def traffic_from_profiles(kernel_tag):
    """HBM bytes per fused pass from committed rocprofv3 counter summaries, if any."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d.get("bytes_per_launch")


def cpu_baseline(p, n_sweeps):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import oracle as O
    f = [np.maximum(t, 1e-10).astype(np.float64) for t in p.init]
    O.sweep(p.model_str, f, p.Y, p.M, p.alpha, p.beta, 1e-10)  # warm-up
    t0 = time.perf_counter()
    for _ in range(n_sweeps):
        f = O.sweep(p.model_str, f, p.Y, p.M, p.alpha, p.beta, 1e-10)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": n_sweeps / dt, "unit": "sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_sweeps} full FP64 sweeps of the same workload after 1 warm-up "
                      f"({dt:.1f} s, numpy einsum on {os.cpu_count()} host CPUs)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method's multi-GPU sharding is described, not built).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2602_02759_amd import datagen
    from paper_2602_02759_amd.nnef import Plan

    n, R = args.n, args.rank
    p = datagen.cp3(args.alpha, args.beta, n=n, R=R)
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(p.Y).to(dev)
    M = torch.from_numpy(p.M).to(dev)
    f = [torch.from_numpy(np.maximum(t, 1e-10)).to(dev) for t in p.init]
    plan = Plan(p.model_str, p.mode_sizes, p.ranks, p.alpha, p.beta, prec=args.prec)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        Yc = torch.empty_like(Y)
        Yc.copy_(Y)
        torch.cuda.synchronize()
        del Yc
    plan.step(Y, M, f, n_sweeps=args.warmup)
    torch.cuda.synchronize()
    plan.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    plan.step(Y, M, f, n_sweeps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    n_pass, pass_ms = plan.timing()
    plan.set_timing(False)
    ms_per_step = ms / args.steps
    N = n * n * n
    L = 3
    has_d = True  # the mask makes D a real contraction
    flops_per_pass = (6 if has_d else 4) * R * N
    avg_pass_s = pass_ms / max(n_pass, 1) / 1e3
    achieved = flops_per_pass / avg_pass_s / 1e12
    traffic = traffic_from_profiles("fused_pass_cp3_256_r32")
    out = {
        "metric": "MU sweeps/s (CP 256^3 R=32, plain FP32)",
        "value": 1e3 / ms_per_step,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"CP 'ir,jr,kr->ijk' {n}^3 R={R}, Poisson counts from "
                               f"Gamma(0.3,1) factors, 20% missing, (alpha,beta)=({args.alpha:g},"
                               f"{args.beta:g}), FP32 contractions",
                   "sweeps_timed": args.steps, "wall_s": wall},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32"],
                     "unit": "TFLOP/s", "frac": achieved / PEAK["fp32"], "traffic": traffic,
                     "kernel": "fused_pass", "flops_per_launch": flops_per_pass,
                     "avg_launch_us": avg_pass_s * 1e6, "launches_timed": n_pass,
                     "alg_bytes_per_launch": N * 5,
                     "alg_GBps": N * 5 / avg_pass_s / 1e9},
    }
    if args.cpu_sweeps > 0:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
