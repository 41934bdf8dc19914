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


PROFILE = os.path.join(ROOT, "profiles", "walk_ba_n1e5_fp32.txt")
KERNEL_SOURCES = ["paper_1904_12759_amd/csrc/walk.hip", "paper_1904_12759_amd/csrc/walk_task.hpp",
                  "paper_1904_12759_amd/csrc/mc_internal.hpp"]


def measured_traffic(profile=PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy), or None when the kernel sources have changed
    since the counters were taken."""
    import hashlib
    try:
        text = open(profile).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    fields = dict(ln.split(":", 1) for ln in text.splitlines()
                  if ":" in ln and not ln.startswith(("#", " ")))
    if fields.get("source_sha256", "").split(" ")[1:2] != [h.hexdigest()]:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"].split()[0])
    except (KeyError, ValueError):
        return None


def measured_valu(profile=PROFILE, sources=KERNEL_SOURCES):
    """The walk kernel's VALU issue from the same committed summary: busy time
    (SQ_ACTIVE_INST_VALU x 4 cycles over 1024 SIMDs at 2.4 GHz) against the launch,
    or None when the kernel sources have changed since."""
    if measured_traffic(profile, sources) is None:
        return None
    import re
    for ln in open(profile).read().splitlines():
        m = re.match(r"valu_busy_estimate: .* = ([0-9.e+]+) cycles = ([0-9.]+) ms of a ([0-9.]+) ms launch",
                     ln)
        if m:
            busy, launch = float(m.group(2)), float(m.group(3))
            return {"busy_ms": busy, "launch_ms": launch, "frac": busy / launch,
                    "source": "rocprofv3 SQ_ACTIVE_INST_VALU"}
    return None


def cpu_baseline(w, seed, nthreads, min_seconds=10.0):
    """The oracle on the host over the same workload (every node, 1e3 walkers each),
    repeated until at least min_seconds of wall time so the rate is not dominated by
    thread start-up; walker-steps per second over all passes."""
    import oracle
    from oracle import Oracle
    oracle.build()
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, seed)
    v = np.asarray(w.v, np.float32).astype(np.float64)
    events = 0
    passes = 0
    t0 = time.perf_counter()
    while True:
        _, _, ev, _ = o.estimate(v, None, w.nwalk, threads=nthreads, counts=True)
        events += int(ev.sum())
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    return dict(value=events / dt, unit="walker-steps/s", cores=nthreads, kind="oracle",
                sample=f"whole workload ({w.a.n} nodes x {w.nwalk} walkers) {passes} times, "
                       f"{dt:.1f} s, {nthreads} threads")


def entries_at_1e3(mc, h, v, idx, pilot: int, target: float = 1e-3, cap: int = 1 << 31,
                   max_passes: int = 4, margin: float = 1.2):
    """Entries/s at a relative standard error target.  A pilot of `pilot` walkers per
    entry estimates sigma_i / x_i; every entry is then run with
    N_i = ceil(margin (sigma_i / (target x_i))^2) walkers (the margin covers the pilot's
    own error on sigma_i, so that one pass usually suffices), all entries in one launch
    (mc_expmv_entries_multi).  Entries whose measured relative error still exceeds the
    target (a pilot underestimates heavy tails) are re-run with N scaled by
    (error / target)^2 * 1.25, up to max_passes.  The time covers every production
    pass; the pilot is not counted."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    idx = np.asarray(idx, np.int64)
    v = h._v(v)                      # device copy once, outside the timed passes
    est, se = h.entries(v, idx, pilot)
    x = est.cpu().numpy()
    sig = se.cpu().numpy() * np.sqrt(pilot)
    need = np.clip(np.ceil(margin * (sig / (target * np.abs(x))) ** 2), 2, cap)
    todo = np.arange(len(idx))
    final_rel = np.zeros(len(idx))
    final_n = np.zeros(len(idx))
    seconds = 0.0
    walkers = 0
    passes = 0
    while len(todo) and passes < max_passes:
        passes += 1
        counts = np.minimum(need[todo], cap).astype(np.int64)
        ti = torch.as_tensor(idx[todo], device=dev)
        e = torch.empty(len(todo), dtype=torch.float64, device=dev)
        s_ = torch.empty(len(todo), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.entries_multi(v, ti, counts, est=e, stderr=s_, sync=False)
        h.sync()
        seconds += time.perf_counter() - t0
        rel = (s_ / e.abs()).cpu().numpy()
        final_rel[todo] = rel
        final_n[todo] = counts
        walkers += int(counts.sum())
        bad = rel > target
        need[todo[bad]] = np.minimum(np.ceil(counts[bad] * (rel[bad] / target) ** 2 * 1.25), cap)
        todo = todo[bad]
    return dict(entries=len(idx), seconds=seconds, entries_per_s=len(idx) / seconds,
                walkers=int(walkers), passes=passes, max_rel_stderr=float(final_rel.max()),
                entries_above_target=int((final_rel > target).sum()),
                final_walkers_max=int(final_n.max()))


def bench_grid2d_entries(mc, seed):
    """2-D Dirichlet Laplacian 32x32, t = 0.1, 16 entries, FP64: entries/s at 1e-3."""
    from paper_1904_12759_amd import workloads as wl
    w = wl.config_grid2d_entries()
    h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed)
    entries_at_1e3(mc, h, w.v, w.idx, 10_000)                       # warm-up
    r = entries_at_1e3(mc, h, w.v, w.idx, 10_000)
    r["workload"] = "grid2d 32x32 Dirichlet, t=0.1, 16 entries, FP64, two-pass (pilot 1e4)"
    return r


def bench_locality(mc, w, seed, steps=10):
    """Kernel time of the benchmark workload with the rows in input order, relabelled
    hot-first (descending exit rate), relabelled with the hottest rows staged in LDS,
    and relabelled with the wave re-sort by current node; then the same variants on
    long walks (the same graph at t = 16, 100 walkers per node).  All variants of a
    workload give bitwise identical results."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    se = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    variants = (("input_order", 0, 0, 0), ("relabel", 1, 0, 0), ("relabel_lds16k", 1, 16384, 0),
                ("relabel_lds64k", 1, 65536, 0), ("relabel_resort1", 1, 0, 1),
                ("relabel_resort4", 1, 0, 4))
    out = {}
    for case, t, nwalk in (("t1", w.t, w.nwalk), ("t16_long_walks", 16.0, 100)):
        ref = None
        res = {}
        for name, relabel, lds, resort in variants:
            h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, t, seed, fp32=True, relabel=relabel,
                           lds_budget=lds, resort_period=resort)
            h.full(v, nwalk, est=est, stderr=se)
            ms = []
            for _ in range(steps):
                h.full(v, nwalk, est=est, stderr=se)
                ms.append(h.stats()["ms"])
            if ref is None:
                ref = est.clone()
            res[name] = dict(kernel_ms=float(np.median(ms)), identical=bool(torch.equal(est, ref)))
            if name == "input_order":
                st = h.stats()
                res["events_per_walker"] = st["events"] / st["walkers"]
            del h
        out[case] = res
    return out


def bench_grid3d(mc, seed, m=256, steps=5):
    """3-D variable-coefficient diffusion 256^3, t = 0.05, full vector with 256
    walkers per node (4.3e9 walkers), FP32 weights: walker-steps/s and roofline."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    t0 = time.perf_counter()
    w = wl.config_grid3d_full(m)
    gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed, fp32=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    se = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    h.full(v, w.nwalk, est=est, stderr=se)
    ms = []
    for _ in range(steps):
        h.full(v, w.nwalk, est=est, stderr=se)
        ms.append(h.stats()["ms"])
    st = h.stats()
    kern = float(np.median(ms))
    achieved = st["alg_bytes"] / (kern / 1e3) / 1e9
    rel = (se / est.abs()).cpu().numpy()
    del h
    return dict(workload=f"grid3d {m}^3 variable coefficient, t=0.05, full vector, "
                         f"{w.nwalk} walkers/node, FP32 weights",
                n=w.a.n, nnz=w.a.nnz, walkers=st["walkers"], events=st["events"],
                jumps=st["jumps"], kernel_ms=kern, walker_steps_per_s=st["events"] / (kern / 1e3),
                roofline_frac=achieved / HBM_PEAK_GBS, achieved_gbs=achieved,
                traffic=measured_traffic(os.path.join(ROOT, "profiles", "walk_grid3d_256_fp32.txt")),
                setup_s=setup, generation_s=gen, median_rel_stderr=float(np.median(rel)))


def bench_batched(mc, seed, runs=5):
    """64 instances in one persistent launch (ER and power-law graphs, n log-uniform in
    [1e3, 1e6], A = adjacency / lambda_max, t ~ U[0.05, 1], v ~ U[0,1]; 32 entries x 1e4
    walkers or the full vector x 64 walkers per node), schedule from the autotuner,
    against the same 64 instances run as separate launches."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    t0 = time.perf_counter()
    ws = wl.batched_instances(count=64)
    gen = time.perf_counter() - t0
    insts = [dict(rowptr=w.a.rowptr, col=w.a.col, val=w.a.val, t=w.t, v=w.v, idx=w.idx,
                  n_walkers=w.nwalk, instance_id=k) for k, w in enumerate(ws)]
    os.environ.pop("MC_EXPMV_TUNE_CACHE", None)
    t0 = time.perf_counter()
    b = mc.MCBatch(insts, seed)
    create_s = time.perf_counter() - t0
    b.run()
    ms = []
    for _ in range(runs):
        b.run()
        ms.append(b.stats()["ms"])
    st = b.stats()
    kern = float(np.median(ms))
    # the same instances as separate handles, one launch each
    hs = [mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed, instance=k)
          for k, w in enumerate(ws)]
    dev = torch.device("cuda", torch.cuda.current_device())
    vs = [torch.as_tensor(w.v, device=dev) for w in ws]
    outs = [torch.empty(len(w.idx) if w.idx is not None else w.a.n, dtype=torch.float64,
                        device=dev) for w in ws]
    idxs = [torch.as_tensor(w.idx, device=dev) if w.idx is not None else None for w in ws]

    def separate():
        for h, w, v, o, ix in zip(hs, ws, vs, outs, idxs):
            if ix is None:
                h.full(v, w.nwalk, est=o, sync=False)
            else:
                h.entries(v, ix, w.nwalk, est=o, sync=False)
        torch.cuda.synchronize()

    separate()
    same = all(torch.equal(outs[k], b.est[k]) for k in range(len(ws)))
    t0 = time.perf_counter()
    for _ in range(runs):
        separate()
    sep_ms = (time.perf_counter() - t0) * 1e3 / runs
    t0 = time.perf_counter()
    for _ in range(runs):
        b.run(sync=False)
    torch.cuda.synchronize()
    b.sync()
    batch_wall_ms = (time.perf_counter() - t0) * 1e3 / runs
    achieved = st["alg_bytes"] / (kern / 1e3) / 1e9
    return dict(workload="64 instances: ER (mean degree 8) and Chung-Lu power-law (gamma 2.5) "
                         "graphs, n log-uniform [1e3, 1e6], A = adjacency/lambda_max, "
                         "t ~ U[0.05,1], 32 entries x 1e4 walkers or full vector x 64/node",
                n_total=int(sum(w.a.n for w in ws)), nnz_total=int(sum(w.a.nnz for w in ws)),
                walkers=st["walkers"], events=st["events"], jumps=st["jumps"],
                kernel_ms=kern, walker_steps_per_s=st["events"] / (kern / 1e3),
                roofline_frac=achieved / HBM_PEAK_GBS, schedule=b.schedule(),
                traffic=measured_traffic(os.path.join(ROOT, "profiles", "walk_batched_64.txt"),
                                         KERNEL_SOURCES + ["paper_1904_12759_amd/csrc/batch.hip"]),
                batch_wall_ms=batch_wall_ms, separate_launches_wall_ms=sep_ms,
                identical_to_separate=bool(same), create_s=create_s, generation_s=gen)


def _ba_learned_case(n, m, gseed):
    """BA(n, m, gseed), A = (0.5/lambda_max) adjacency, v ~ U[0,1] (seed 2); 1024 entries
    (the 256 highest-degree nodes and 768 uniform ones, seed 3)."""
    from paper_1904_12759_amd import workloads as wl
    g = wl.ba_graph(n, m, gseed)
    lam = wl.lambda_max(g)
    a = wl.scaled(g, 0.5 / lam)
    v = wl.uniform_v(a.n, 2)
    deg = np.diff(a.rowptr)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.argsort(-deg)[:256], rng.choice(a.n, 768, replace=False)]))
    return a, v, idx, lam


def _steps_to_target(a, v, idx, bias, events_per_walker, t=1.0, target=1e-3):
    """Walker-steps for a relative standard error of `target` at every entry, from the
    exact per-entry variance: x = exp(tA) v and, by Feynman-Kac with the jump factors
    e^{-b}, E[f^2] = exp(tG) v^2 with G_ij = a_ij e^{-b_ij}, G_ii = 2 d~_i - r~_i."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    deg = np.diff(a.rowptr)
    rows = np.repeat(np.arange(a.n), deg)
    b = np.zeros(a.nnz) if bias is None else np.asarray(bias, np.float64)
    at = a.val * np.exp(b)
    rt = np.bincount(rows, weights=at, minlength=a.n)
    r = np.bincount(rows, weights=a.val, minlength=a.n)
    gm = sp.csr_matrix((a.val * np.exp(-b), a.col, a.rowptr), shape=(a.n, a.n))
    gm = gm + sp.diags(2 * (r + (rt - r)) - rt)         # d = r (no diagonal in A)
    m2 = sla.expm_multiply((t * gm).tocsr(), v * v)
    x = sla.expm_multiply((t * a.to_scipy()).tocsr(), v)
    xi = x[idx]
    var = np.maximum(m2[idx] - xi * xi, 0)
    return float((var / (target * xi) ** 2).sum() * events_per_walker)


def bench_learned(mc, seed, n=1_000_000, m=4):
    """Learned vs plain proposal on BA(n=1e6, m=4), t = 1: walker-steps to 1e-3 relative
    standard error for the plain and the learned walk from exact per-entry variances, and
    the learned walk's measured entries/s.  The network is trained on the graph of seed 1
    and also applied, unchanged, to a held-out graph of seed 2 (features computed there)."""
    import torch
    t_gen = time.perf_counter()
    a, v, idx, lam = _ba_learned_case(n, m, 1)
    t_gen = time.perf_counter() - t_gen

    def events_per_walker(h, vv, ii):
        h.entries(vv, ii, 1 << 14)      # plain, or tilted once a proposal is installed
        st = h.stats()
        return st["events"] / st["walkers"]

    h = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, seed)
    ev_plain = events_per_walker(h, v, idx)
    rep = h.learn_proposal(v, pilot_walkers=256, steps=400, batch=1 << 16, lr=3e-3, seed=1)
    bias = h.get_proposal().cpu().numpy()
    ev_learn = events_per_walker(h, v, idx)
    steps_p = _steps_to_target(a, v, idx, None, ev_plain)
    steps_l = _steps_to_target(a, v, idx, bias, ev_learn)
    prod = entries_at_1e3(mc, h, v, idx, 10_000)
    out = dict(workload=f"BA n={n} m={m} seed 1, A=(0.5/lambda_max)*adjacency "
                        f"(lambda_max={lam:.6g}), t=1, v~U[0,1], {len(idx)} entries "
                        "(256 highest degree + uniform)", generation_s=t_gen,
               walker_steps_to_1e3_plain_exact=steps_p,
               walker_steps_to_1e3_learned_exact=steps_l,
               gain_walker_steps=steps_p / steps_l if steps_l > 0 else None,
               events_per_walker_plain=ev_plain, events_per_walker_learned=ev_learn,
               learned_entries_per_s_at_1e3=prod["entries_per_s"],
               learned_production_s=prod["seconds"],
               learned_max_rel_stderr=prod["max_rel_stderr"],
               train=dict(initial_loss=rep["initial_loss"], final_loss=rep["final_loss"],
                          steps=rep["steps"], pilot_ms=rep["pilot_ms"], train_ms=rep["train_ms"]))
    del h
    # held-out graph: same network, features of the new graph
    a2, v2, idx2, lam2 = _ba_learned_case(n, m, 2)
    h2 = mc.MCExpmv(a2.rowptr, a2.col, a2.val, 1.0, seed)
    ev_plain2 = events_per_walker(h2, v2, idx2)
    net = mc.MLP(h2, seed=1)
    net.set_params(rep["params"])
    dev = torch.device("cuda", torch.cuda.current_device())
    feats2 = h2.features(torch.as_tensor(v2, device=dev))
    bias2 = net.forward(feats2)
    h2.set_proposal(bias2)
    ev_learn2 = events_per_walker(h2, v2, idx2)
    steps_p2 = _steps_to_target(a2, v2, idx2, None, ev_plain2)
    steps_l2 = _steps_to_target(a2, v2, idx2, bias2.cpu().numpy(), ev_learn2)
    prod2 = entries_at_1e3(mc, h2, v2, idx2, 10_000)
    out["held_out"] = dict(
        workload=f"BA n={n} m={m} seed 2 (lambda_max={lam2:.6g}), same recipe; network "
                 "trained on seed 1, not retrained",
        walker_steps_to_1e3_plain_exact=steps_p2, walker_steps_to_1e3_learned_exact=steps_l2,
        gain_walker_steps=steps_p2 / steps_l2 if steps_l2 > 0 else None,
        learned_entries_per_s_at_1e3=prod2["entries_per_s"],
        learned_max_rel_stderr=prod2["max_rel_stderr"])
    net.close()
    return out


def bench_forward_tc(mc, seed, n=1_000_000, m=1_000_000, steps=5):
    """Total communicability TC = (1, e^A 1) (Eq. (TC)) of a small-world network
    (Newman-Watts ring with shortcuts, mean degree 2.4, n = 1e6) by forward walks
    (Theorem 2, Algorithm 2) with M = 1e6 walkers, in STRANG mode with the paper's
    dt = 0.03125 (the setting of its Tables 0 and 00) and in EXACT mode; against the
    exact TC from expm_multiply."""
    import torch
    import scipy.sparse.linalg as sla
    from paper_1904_12759_amd import workloads as wl
    t0 = time.perf_counter()
    a = wl.small_world(n, 0.2, 1)
    gen = time.perf_counter() - t0
    exact = float(sla.expm_multiply(a.to_scipy().tocsr(), np.ones(a.n)).sum())
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.ones(a.n, dtype=torch.float64, device=dev)
    out = dict(workload=f"small world (Newman-Watts, p=0.2) n={n}, mean degree "
                        f"{a.nnz / a.n:.3f}, A = adjacency, t = 1, v = 1, M = {m} walkers",
               tc_exact=exact, generation_s=gen)
    for name, mode in (("strang_dt_0.03125", mc.STRANG), ("exact", mc.EXACT)):
        h = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, seed, mode=mode, dt=0.03125)
        tot = torch.empty(2, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        h.forward(v, m, total=tot, total_only=True)        # includes the symmetry check
        first = time.perf_counter() - t0
        ms = []
        for _ in range(steps):
            h.forward(v, m, total=tot, total_only=True)
            ms.append(h.stats()["ms"])
        st = h.stats()
        tc, tse = tot.cpu().numpy().tolist()
        out[name] = dict(ms_per_tc=float(np.median(ms)), first_call_s=first, tc=tc,
                         tc_n=tc / a.n, rel_stderr=tse / abs(tc),
                         rel_err_vs_exact=(tc - exact) / exact,
                         events=st["events"], jumps=st["jumps"],
                         walker_steps_per_s=st["events"] / (float(np.median(ms)) / 1e3))
        del h
    return out


def bench_isim(mc, seed, ms=(100_000, 1_000_000, 10_000_000), per_node=(1_000, 10_000, 100_000)):
    """Ranking study (Sec. 6, the isim table): small-world networks n = 1000 and 10000
    (Newman-Watts, p = 0.2), A = adjacency, t = 1, v = 1, so the full vector is every
    node's total subgraph communicability.  Forward walks (Algorithm 2), STRANG with the
    paper's dt = 0.03125, M walkers in total, and backward walks (Algorithm 1) with M
    walkers per node; the Monte Carlo vector ranked against the exact one
    (expm_multiply) by isim at K = n and K = n/10 (mc_isim on the GPU), with the
    normalised total communicability TC_n = TC / n."""
    import torch
    import scipy.sparse.linalg as sla
    from paper_1904_12759_amd import workloads as wl
    dev = torch.device("cuda", torch.cuda.current_device())
    out = {}
    for n in (1000, 10_000):
        a = wl.small_world(n, 0.2, 1)
        exact = sla.expm_multiply(a.to_scipy().tocsr(), np.ones(a.n))
        ex = torch.as_tensor(exact, device=dev)
        v = torch.ones(a.n, dtype=torch.float64, device=dev)
        h = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, seed, mode=mc.STRANG, dt=0.03125)
        rows = {}
        for m in ms:
            est, se, tot = h.forward(v, m)
            tc = float(tot[0].item())
            rows[str(m)] = dict(isim_100=mc.isim(est, ex), isim_10=mc.isim(est, ex, n // 10),
                                tc_n=tc / n, tc_n_exact=float(exact.sum()) / n,
                                tc_n_rel_stderr=float(tot[1].item()) / abs(tc),
                                max_rel_err=float(np.max(np.abs(est.cpu().numpy() - exact) / exact)))
        # the other reading of the sample size: M backward walkers per node (Algorithm 1)
        back = {}
        for m in per_node:
            est, se = h.full(v, m)
            back[str(m)] = dict(isim_100=mc.isim(est, ex), isim_10=mc.isim(est, ex, n // 10),
                                max_rel_err=float(np.max(np.abs(est.cpu().numpy() - exact) / exact)),
                                ms=h.stats()["ms"])
        out[f"n{n}"] = dict(forward_total_walkers=rows, backward_walkers_per_node=back)
        del h
    out["workload"] = ("small world (Newman-Watts, p=0.2), A = adjacency, t = 1, v = 1; forward "
                       "walks, STRANG dt = 0.03125; isim against expm_multiply")
    return out


def bench_splitting(mc, seed, m_total=4_000_000, m_entry=1_000_000):
    """Splitting study (Sec. 5, Figs. 2-3): small-world networks n = 100 and 1000
    (Newman-Watts, mean degree 2.4), A = adjacency, t = 1, v = 1, dt = 1/2 .. 1/64.  Per
    dt the exact errors of the Strang and Lie products (dense) for the total
    communicability and for entry 0, the errors of the GPU estimates in STRANG and LIE
    mode (forward walks for the total, M = 4e6; backward walks for entry 0, 1e6 walkers)
    with their standard errors, and the leading Strang term |(1, D L D 1)| dt^2."""
    import torch
    import scipy.linalg as sla
    from paper_1904_12759_amd import workloads as wl

    def split_parts(a):
        off = a - np.diag(np.diag(a))
        return np.diag(a) + off.sum(1), np.diag(off.sum(1)) - off     # d, L

    def strang(a, nsteps, x):        # (e^{dt D/2} e^{-dt L} e^{dt D/2})^N x
        d, lap = split_parts(a)
        dt = 1.0 / nsteps
        h = np.exp(dt * d / 2)
        step = h[:, None] * sla.expm(-dt * lap) * h[None, :]
        for _ in range(nsteps):
            x = step @ x
        return x

    def lie(a, nsteps, x):           # (e^{-dt L} e^{dt D})^N x
        d, lap = split_parts(a)
        dt = 1.0 / nsteps
        step = sla.expm(-dt * lap) * np.exp(dt * d)[None, :]
        for _ in range(nsteps):
            x = step @ x
        return x

    dev = torch.device("cuda", torch.cuda.current_device())
    dts = [0.5, 0.25, 0.125, 0.0625, 0.03125, 0.015625]
    out = dict(dts=dts)
    for n in (100, 1000):
        w = wl.small_world(n, 0.2, 3)
        a = w.to_dense()
        one = np.ones(n)
        exact = sla.expm(a) @ one
        dvec, lap = split_parts(a)
        lead = abs(one @ (dvec * (lap @ (dvec * one))))
        rec = dict(tc_exact=float(exact.sum()), x0_exact=float(exact[0]),
                   strang_lead_coef=float(lead))
        v = torch.ones(n, dtype=torch.float64, device=dev)
        for name, mode, prod in (("strang", mc.STRANG, strang), ("lie", mc.LIE, lie)):
            r = dict(tc_split_err=[], x0_split_err=[], tc_mc_err=[], tc_mc_se=[], x0_mc_err=[],
                     x0_mc_se=[])
            for dt in dts:
                nsteps = int(round(1 / dt))
                p = prod(a, nsteps, one)
                r["tc_split_err"].append(float(p.sum() - exact.sum()))
                r["x0_split_err"].append(float(p[0] - exact[0]))
                h = mc.MCExpmv(w.rowptr, w.col, w.val, 1.0, seed, mode=mode, dt=dt)
                _, _, tot = h.forward(v, m_total, total_only=True)
                tc, tse = tot.cpu().numpy().tolist()
                e, se = h.entries(v, [0], m_entry)
                r["tc_mc_err"].append(tc - float(exact.sum()))
                r["tc_mc_se"].append(tse)
                r["x0_mc_err"].append(e.item() - float(exact[0]))
                r["x0_mc_se"].append(se.item())
                del h
            fit = lambda errs: float(np.polyfit(np.log(dts), np.log(np.abs(errs)), 1)[0])
            r["tc_split_order"] = fit(r["tc_split_err"])
            r["x0_split_order"] = fit(r["x0_split_err"])
            rec[name] = r
        out[f"n{n}"] = rec
    return out


# first-jump conditioning only where the start node keeps its walkers with
# probability >= 1/2 (r t <= ln 2)
HYBRID_RT = 0.6931471805599453


def bench_conditioning(mc, seed, steps=10):
    """First-jump conditioning against the plain walk: on the main BA n=1e5 workload
    (full vector, 1000 walkers per node, FP32) the kernel time and the per-node
    variance, combined as the work-normalised gain (var_plain t_plain) /
    (var_cond t_cond), median over nodes; and entries/s at 1e-3 on the grid2d
    32x32 entries workload (FP64), both walks."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    out = {}
    w = wl.config_ba_full()
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    res = {}
    for name, cond, theta in (("plain", False, np.inf), ("cond", True, np.inf),
                              ("hybrid", True, HYBRID_RT)):
        h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed, fp32=True, cond=cond,
                       cond_max_rt=theta)
        est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
        se = torch.empty(w.a.n, dtype=torch.float64, device=dev)
        h.full(v, w.nwalk, est=est, stderr=se)
        ms = []
        for _ in range(steps):
            h.full(v, w.nwalk, est=est, stderr=se)
            ms.append(h.stats()["ms"])
        st = h.stats()
        res[name] = (float(np.median(ms)), (se * se).cpu().numpy(), st["events"])
        del h
    deg = np.diff(w.a.rowptr)
    out["ba_full"] = dict(
        workload="BA n=1e5 m=3, full vector, 1000 walkers/node, FP32 weights",
        hybrid_cond_max_rt=HYBRID_RT)
    for name in ("cond", "hybrid"):
        gain = (res["plain"][1] * res["plain"][0]) / np.maximum(res[name][1] * res[name][0], 1e-300)
        # total work to bring every node to the same standard error: sum of variances x time
        total = (res["plain"][1].sum() * res["plain"][0]) / (res[name][1].sum() * res[name][0])
        out["ba_full"][name] = dict(
            kernel_ms=res[name][0], events=res[name][2],
            median_work_normalised_gain=float(np.median(gain)),
            median_gain_degree_3=float(np.median(gain[deg == 3])),
            median_gain_top_1pct_degree=float(np.median(gain[deg >= np.quantile(deg, 0.99)])),
            total_work_gain=float(total))
    out["ba_full"]["kernel_ms_plain"] = res["plain"][0]
    g2 = wl.config_grid2d_entries()
    for name, cond in (("plain", False), ("cond", True)):
        h = mc.MCExpmv(g2.a.rowptr, g2.a.col, g2.a.val, g2.t, seed, cond=cond)
        entries_at_1e3(mc, h, g2.v, g2.idx, 10_000)                       # warm-up
        r = entries_at_1e3(mc, h, g2.v, g2.idx, 10_000)
        out[f"grid2d_entries_at_1e3_{name}"] = dict(entries_per_s=r["entries_per_s"],
                                                    walkers=r["walkers"],
                                                    max_rel_stderr=r["max_rel_stderr"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every extra measurement (same as --extras none)")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extra measurements after the main step: "
                         "locality, entries, learned, grid3d, batched, forward, cond, splitting, isim; "
                         "'all' or 'none'")
    ap.add_argument("--seed", type=int, default=12759)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (steps times), "
                         "the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard walkers by start node, which is not implemented)",
              file=sys.stderr)
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
            "traffic": measured_traffic(),
        },
        # the tables are cache resident (traffic above is a few % of the algorithmic
        # bytes): the kernel is bound by vector-ALU issue, which this reports
        "valu_issue": measured_valu(),
    }
    names = ["locality", "entries", "learned", "grid3d", "batched", "forward", "cond", "splitting",
             "isim"]
    extras = [] if args.no_extras or args.extras == "none" else \
        names if args.extras == "all" else [x for x in args.extras.split(",") if x]
    unknown = [x for x in extras if x not in names]
    if unknown:
        print(f"bench.py: unknown extras {unknown}; choose from {names}", file=sys.stderr)
        sys.exit(2)
    if "locality" in extras:
        log("bench: locality variants")
        out["locality"] = bench_locality(mc, w, args.seed)
    if "entries" in extras:
        log("bench: entries/s at 1e-3 (grid2d)")
        out["entries_at_1e3"] = bench_grid2d_entries(mc, args.seed)
    if "learned" in extras:
        log("bench: learned vs plain (BA n=1e6 m=4)")
        out["learned_vs_plain"] = bench_learned(mc, args.seed)
    if "grid3d" in extras:
        log("bench: grid3d 256^3")
        out["grid3d_256"] = bench_grid3d(mc, args.seed)
    if "batched" in extras:
        log("bench: batched 64 instances")
        out["batched_64"] = bench_batched(mc, args.seed)
    if "forward" in extras:
        log("bench: forward total communicability (small world n=1e6)")
        out["forward_tc"] = bench_forward_tc(mc, args.seed)
    if "cond" in extras:
        log("bench: first-jump conditioning vs plain")
        out["conditioning"] = bench_conditioning(mc, args.seed)
    if "splitting" in extras:
        log("bench: splitting study (small world n=100, 1000)")
        out["splitting"] = bench_splitting(mc, args.seed)
    if "isim" in extras:
        log("bench: ranking study (small world n=1000, 10000)")
        out["isim"] = bench_isim(mc, args.seed)
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
