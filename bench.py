"""Benchmark of the SFT/ASFT kernel-integral Morlet transform on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line. A step is one pass of the transform over the workload's batch,
with inputs resident in HBM. The dominant kernel is timed with HIP events on the
stream it is launched on, and its algorithmic bytes per launch give the roofline figure.
The FP64 oracle is timed on the host cores on a bounded sample for the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="paper_scale", choices=["paper_scale"])
    ap.add_argument("--mode", default="asft", choices=["sft", "asft"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return ap.parse_args()


def cpu_baseline_paper_scale(x, info, mode):
    """FP64 oracle (numpy kernel-integral recurrences) on the same signal, one transform."""
    from oracle import morlet_oracle as O
    p = O.plan_morlet(8192.0, 6.0 / 8192.0, 6, 32768, mode=mode, n0=info["n0"] if mode == "asft" else None,
                      P_S=info["P_S"])
    xd = x.astype(np.float64)
    O.forward(xd, p)                     # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        O.forward(xd, p)
        reps += 1
        el = time.perf_counter() - t0
        if el > 10.0 or reps >= 50:
            break
    per = el / reps
    return {"value": len(x) / per / 1e9, "unit": "Gsamples*scales/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full transforms of the N=102400 signal (6 terms, numpy float64, one thread)"}


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2110_11866_amd as M
    import workloads

    dev = torch.device("cuda:0")
    N, sigma, K, L = 102400, 8192.0, 6, 32768
    x = workloads.paper_scale_signal(N)
    xt = torch.from_numpy(x).to(dev)
    plan = M.MorletPlan(N, sigma, 6.0 / sigma, K, L, mode=args.mode)
    info = plan.info()
    out = torch.empty(N, dtype=torch.complex64, device=dev)
    ws = plan.workspace(dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.forward(xt, out=out, ws=ws)
    torch.cuda.synchronize()

    # timed region: K steps, bracketed by synchronisation
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        plan.forward(xt, out=out, ws=ws)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    kern_ms_avg = float(np.mean(kern_ms))
    ms_per_step = wall * 1e3 / args.steps

    samples_scales = N * 1
    bytes_per_launch = N * 4 + N * 8        # float32 in, complex64 out
    achieved = bytes_per_launch / (kern_ms_avg * 1e-3) / 1e9
    line = {
        "metric": "Gsamples*scales/s (ASFT-scan Morlet transform)",
        "value": samples_scales / (ms_per_step * 1e-3) / 1e9,
        "unit": "Gsamples*scales/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper_scale: N=102400, sigma=8192, xi=6/sigma, K=6, L=32768, "
                               f"{args.mode}, float32 in, complex64 out",
                   "P_S": info["P_S"], "n0": info["n0"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "kernel_us": kern_ms_avg * 1e3,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_paper_scale(x, info, args.mode)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
