#!/usr/bin/env python3
"""Benchmark of the Monte Carlo exp(tA)v estimator on one MI355X.

Workload (one "step" = one pass of the whole path over the batch): the full
vector exp(A) 1 of a Barabasi-Albert graph, n = 1e5, m = 3 (seed 1),
A = (0.5 / lambda_max) * adjacency, t = 1, 1000 walkers per node, FP32 weights
and FP64 reductions (EXACT weights, the dt -> 0 limit of the splittings).
Inputs are synthetic and already resident in HBM when timing starts.

Prints ONE JSON line with walker-steps/s (holding intervals per second), the
roofline position of the walk kernel and the CPU oracle's rate on the host.
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

METRIC = "walker-steps/s and entries/s at 1e-3 rel err; learned vs plain proposal"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, seed, nthreads):
    """The oracle on the host: the same workload (every node, 1e3 walkers each)."""
    import oracle
    from oracle import Oracle
    oracle.build()
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, seed)
    v = np.asarray(w.v, np.float32).astype(np.float64)
    t0 = time.perf_counter()
    _, _, ev, _ = o.estimate(v, None, w.nwalk, threads=nthreads, counts=True)
    dt = time.perf_counter() - t0
    return dict(value=float(ev.sum()) / dt, unit="walker-steps/s", cores=nthreads,
                kind="oracle",
                sample=f"whole workload: {w.a.n} nodes x {w.nwalk} walkers, {dt:.2f} s, "
                       f"{nthreads} threads")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--seed", type=int, default=12759)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (steps times), "
                         "the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(walkers shard by start node; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1904_12759_amd as mc
    from paper_1904_12759_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "launches": args.steps}), flush=True)
        return
    log("bench: building workload")
    w = wl.config_ba_full()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log("bench: creating handle")
    t0 = time.perf_counter()
    h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, args.seed, fp32=True,
                   stream=stream.cuda_stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    se = torch.empty(w.a.n, dtype=torch.float64, device=dev)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        h.full(v, w.nwalk, est=est, stderr=se, sync=False)
    h.sync()
    st = h.stats()

    log(f"bench: timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        h.full(v, w.nwalk, est=est, stderr=se, sync=False)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.sync()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ms_per_step = wall * 1e3 / args.steps
    st = h.stats()
    events = st["events"]
    value = events / (ms_per_step / 1e3)
    achieved = st["alg_bytes"] / (kern_ms / 1e3) / 1e9
    e_np = est.cpu().numpy()
    s_np = se.cpu().numpy()
    rel = s_np / np.abs(e_np)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 weights / f64 time and sums",
        "data": "synthetic",
        "config": {
            "workload": "BA n=1e5 m=3 seed 1, A=(0.5/lambda_max)*adjacency, t=1, v=1, "
                        "full vector exp(tA)v, 1000 walkers/node, EXACT weights, FP32 weights",
            "n": w.a.n, "nnz": w.a.nnz, "walkers": st["walkers"], "events_per_step": events,
            "jumps_per_step": st["jumps"], "lambda_max": w.note,
        },
        "walkers_per_s": st["walkers"] / (ms_per_step / 1e3),
        "kernel_ms": kern_ms,
        "setup_ms": setup_s * 1e3,
        "median_rel_stderr": float(np.median(rel)),
        "max_rel_stderr": float(np.max(rel)),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
        },
    }
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        try:
            nthreads = len(os.sched_getaffinity(0))
        except AttributeError:
            nthreads = os.cpu_count() or 1
        out["cpu_baseline"] = cpu_baseline(w, args.seed, nthreads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
