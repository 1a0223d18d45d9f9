#!/usr/bin/env python3
"""Throughput of exact VRP-RPD makespan evaluation on one MI355X.

Workload (the full-scale configuration): one instance with n = 1000 customers,
m = 10 vehicles, capacity k = 10, R = 100 resources, processing times
U_int[1,20] * floor(mean depot distance / 10); synthetic TSPLIB-shaped points
(integer, uniform in [0,1000]^2, EUC_2D rounding).  A step evaluates a batch of
65,536 explicit candidate solutions (random drop-before-pickup linear
extensions spread over the vehicles, then renamed customers so that all
65,536 are distinct), all resident in HBM before the timed region.

Prints one JSON line.  The CPU baseline is the oracle (single-threaded C)
timed on a bounded sample of the same candidates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact makespan evals/sec at n=1000; wall time to oracle-best makespan"
HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(B, seed=3003):
    import synth
    inst = synth.make_instance(1000, 10, 10, 100, "1R20d10", seed=seed)
    pool_ops, pool_rt = synth.random_candidates(inst, 1024, seed=seed + 1)
    ops, rt = synth.relabel_candidates(pool_ops, pool_rt, inst.n, B, seed=seed + 2)
    return inst, ops, rt


def cpu_baseline(inst, ops, rt, seconds):
    import oracle
    oracle.lib()
    done, t0, i = 0, time.perf_counter(), 0
    chunk = 1024
    while time.perf_counter() - t0 < seconds and i < len(ops):
        oracle.eval_batch(inst, ops[i:i + chunk], rt[i:i + chunk])
        done += min(chunk, len(ops) - i)
        i += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of the {len(ops)} candidates, single-threaded C oracle, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_23685_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P.load()
    B, K, W = args.batch, args.steps, args.warmup
    log(f"generating workload B={B}")
    inst, ops, rt = make_workload(B)
    S = P.InstanceSet([inst])
    d_ops = torch.from_numpy(ops).cuda()
    d_rt = torch.from_numpy(rt).cuda()
    mk = torch.empty(B, dtype=torch.int32, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        P.vrprpd_eval(S, d_ops, d_rt, makespan=mk, status=st, stream=stream)

    log(f"warmup {W}")
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    feasible = float((st == 0).float().mean().item())

    log(f"timing {K} steps")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    value = B * K / wall
    bytes_per_eval = 2 * 2 * inst.n + 2 * inst.m + 4 + 4
    achieved = bytes_per_eval * B / (kern_ms * 1e-3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "vrprpd_eval, n=1000 customers, m=10 vehicles, k=10, R=100, "
                        "p=U_int[1,20]*floor(dbar/10), 65,536 explicit candidates per step",
            "n": inst.n, "m": inst.m, "k": inst.k, "R": inst.R, "batch": B,
            "feasible_fraction": feasible,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": None,
            "kernel": "eval_kernel", "kernel_ms": kern_ms,
            "bytes_per_eval": bytes_per_eval,
        },
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(inst, ops, rt, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
