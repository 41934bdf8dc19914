#!/usr/bin/env python3
"""Benchmark of the Monte Carlo exp(tA)v estimator on one MI355X.

Workload (one "step" = one pass of the whole path over the batch): the full
vector exp(tA) v of the 3-D variable-coefficient diffusion operator on a 256^3
grid (n = 16.7M, 7-point stencil, cell coefficients log-uniform in [0.1, 10],
harmonic-mean faces, Dirichlet), t = 0.05, v = Gaussian bump + U[0,1] noise,
256 walkers per node (4.3e9 walkers), FP32 weights with FP64 time and sums
(EXACT weights, the dt -> 0 limit of the splittings).  Inputs are synthetic and
already resident in HBM when timing starts.

Prints ONE JSON line with walker-steps/s (holding intervals per second), the
roofline position of the walk kernel and the CPU oracle's rate on the host;
the other benchmark configurations follow as extra keys.
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
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one full-rate 32-bit
# operation per lane per cycle; a wave64 instruction occupies a SIMD 4 cycles)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic VALU work per walker-step: the one Philox4x32-10 call that defines
# the step's random numbers, 10 rounds of two 32x32 -> 64-bit products and two
# three-input XORs each (the key schedule is wave-uniform, on the scalar unit)
PHILOX_LANE_OPS = 40


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1904_12759_amd/csrc/walk.hip", "paper_1904_12759_amd/csrc/walk_task.hpp",
                  "paper_1904_12759_amd/csrc/mc_internal.hpp"]
PROFILE = os.path.join(ROOT, "profiles", "walk_grid3d_256_fp32.txt")
PROFILE_BA = os.path.join(ROOT, "profiles", "walk_ba_n1e5_fp32.txt")
PROFILE_BATCH = os.path.join(ROOT, "profiles", "walk_batched_64.txt")
BATCH_SOURCE = "paper_1904_12759_amd/csrc/batch.hip"


def _profile_fields(profile, sources):
    """key: value lines of a committed rocprofv3 summary, or None when the kernel
    sources have changed since the counters were taken (source_sha256)."""
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
    return fields


def _num(fields, key):
    try:
        return float(fields[key].split()[0])
    except (KeyError, ValueError, TypeError, AttributeError, IndexError):
        return None


def measured_traffic(profile=PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 summary (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy), or None when the kernel sources have changed
    since the counters were taken."""
    f = _profile_fields(profile, sources)
    return None if f is None else _num(f, "traffic_bytes_per_launch")


def measured_counters(profile=PROFILE, sources=KERNEL_SOURCES):
    """The walk kernel's SQ / L2 figures from the same committed summary (None when
    the sources have changed): VALU busy time (SQ_ACTIVE_INST_VALU x 4 cycles over
    1024 SIMDs at 2.4 GHz) against the profiled launch, VALU instructions per
    walker-step, mean occupancy and L2 hit rate."""
    f = _profile_fields(profile, sources)
    if f is None:
        return None
    out = {"source": os.path.relpath(profile, ROOT)}
    for key in ("avg_duration_ms", "valu_busy_ms", "valu_busy_frac", "valu_lane_instr_per_step",
                "occupancy_waves_per_simd", "l2_hit_rate"):
        out[key] = _num(f, key)
    return out


def alu_roofline(events, kern_ms, traffic):
    """The walk is bound by vector-ALU issue (its tables are reused from cache).
    achieved = algorithmic VALU work (PHILOX_LANE_OPS per walker-step) per launch
    / the launch's duration, against the VALU issue peak."""
    achieved = events * PHILOX_LANE_OPS / (kern_ms / 1e3) / 1e12
    peak = VALU_PEAK_LANE_OPS / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "T lane-op/s (VALU; 40 lane-ops of Philox4x32-10 per walker-step)",
            "frac": achieved / peak, "traffic": traffic}


def gather_bytes_lower_bound(k, jumps, fp32, slot_bytes=12):
    """Table and vector bytes a walk must read at least, with no reuse between
    entries: once per entry its start row record (16 B), d and v; per jump the
    slot record and the destination's row record and d."""
    wb = 4 if fp32 else 8
    return k * (16 + 2 * wb) + jumps * (slot_bytes + 16 + wb)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(o, v, idx, nwalk, threads, min_seconds):
    events = 0
    passes = 0
    t0 = time.perf_counter()
    while True:
        _, _, ev, _ = o.estimate(v, idx, nwalk, threads=threads, counts=True)
        events += int(ev.sum())
        passes += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            return events / dt, passes, dt, events / passes


def cpu_baseline(w, seed, nthreads, gpu_events, min_seconds=10.0):
    """The oracle (plain C, FP64, unchanged for this) on the host: all cores on a 1%
    sample of the start nodes (every 100th node, all its walkers), single-threaded on
    a 0.1% sample (every 1000th node); each repeated until min_seconds (the
    single-threaded leg min_seconds / 2) have passed.  Walker-steps per second of
    the sample; the whole workload's time is extrapolated from the rate."""
    import oracle
    from oracle import Oracle
    oracle.build()
    t0 = time.perf_counter()
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, seed)
    create_s = time.perf_counter() - t0
    v = np.asarray(w.v, np.float32).astype(np.float64)
    idx1 = np.arange(0, w.a.n, 100, dtype=np.int64)
    idx01 = np.arange(0, w.a.n, 1000, dtype=np.int64)
    rate, passes, dt, ev_pass = _oracle_rate(o, v, idx1, w.nwalk, nthreads, min_seconds)
    rate1, passes1, dt1, _ = _oracle_rate(o, v, idx01, w.nwalk, 1, min_seconds / 2)
    o.close()
    ev_walker = ev_pass / (len(idx1) * w.nwalk)
    return dict(value=rate, unit="walker-steps/s", cores=nthreads, kind="oracle",
                sample=f"1% of the start nodes (every 100th: {len(idx1)} nodes x {w.nwalk} "
                       f"walkers, {ev_walker:.4f} steps per walker) {passes} times in "
                       f"{dt:.1f} s on {nthreads} threads",
                cpu_model=cpu_model(), single_thread_value=rate1,
                single_thread_sample=f"0.1% of the start nodes (every 1000th: {len(idx01)} "
                                     f"nodes) {passes1} times in {dt1:.1f} s, 1 thread",
                extrapolated_full_workload_s=gpu_events / rate,
                extrapolated_full_workload_s_single_thread=gpu_events / rate1,
                oracle_setup_s=create_s)


def entries_at_1e3(mc, h, v, idx, pilot: int, target: float = 1e-3, cap: int = 1 << 31,
                   max_passes: int = 4, margin: float = 1.2, exact=None, min_walkers: int = 2):
    """Entries/s at a relative standard error target (the error model of Sec. 5).  A
    pilot of `pilot` walkers per entry estimates sigma_i / x_i; every entry is then run
    with N_i = ceil(margin (sigma_i / (target x_i))^2) walkers (the margin covers the
    pilot's own error on sigma_i, so that one pass usually suffices), all entries in
    one launch (mc_expmv_entries_multi).  Entries whose measured relative error still
    exceeds the target (a pilot underestimates heavy tails) are re-run with N scaled
    by (error / target)^2 * 1.25, up to max_passes.  entries_per_s counts every
    production pass; entries_per_s_with_pilot adds the pilot.  With `exact` (the
    deterministic values of the entries) the achieved errors are reported too.
    min_walkers floors each entry's production count (the lattice's standard error
    needs several replicates to be an estimate at all)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    idx = np.asarray(idx, np.int64)
    v = h._v(v)                      # device copy once, outside the timed passes
    ti_all = torch.as_tensor(idx, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, se = h.entries(v, ti_all, pilot)
    pilot_s = time.perf_counter() - t0
    x = est.cpu().numpy()
    sig = se.cpu().numpy() * np.sqrt(pilot)
    need = np.clip(np.ceil(margin * (sig / (target * np.abs(x))) ** 2), min_walkers, cap)
    todo = np.arange(len(idx))
    final_rel = np.zeros(len(idx))
    final_n = np.zeros(len(idx))
    final_est = np.zeros(len(idx))
    final_se = np.zeros(len(idx))
    seconds = 0.0
    walkers = 0
    passes = 0
    rerun = []
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
        en, sn = e.cpu().numpy(), s_.cpu().numpy()
        rel = sn / np.abs(en)
        final_rel[todo] = rel
        final_n[todo] = counts
        final_est[todo] = en
        final_se[todo] = sn
        walkers += int(counts.sum())
        bad = rel > target
        need[todo[bad]] = np.minimum(np.ceil(counts[bad] * (rel[bad] / target) ** 2 * 1.25), cap)
        todo = todo[bad]
        if passes == 1:
            rerun = [int(i) for i in todo]
    out = dict(entries=len(idx), seconds=seconds, entries_per_s=len(idx) / seconds,
               pilot_walkers_per_entry=pilot, pilot_s=pilot_s,
               entries_per_s_with_pilot=len(idx) / (seconds + pilot_s),
               walkers=int(walkers), passes=passes, rerun_after_first_pass=rerun,
               max_rel_stderr=float(final_rel.max()),
               entries_above_target=int((final_rel > target).sum()),
               final_walkers_max=int(final_n.max()))
    if exact is not None:
        ex = np.asarray(exact, np.float64)
        err = np.abs(final_est - ex) / np.abs(ex)
        z = (final_est - ex) / np.maximum(final_se, 1e-300)
        out.update(achieved_max_rel_err=float(err.max()),
                   achieved_median_rel_err=float(np.median(err)),
                   achieved_frac_within_1e3=float(np.mean(err <= target)),
                   achieved_frac_within_3e3=float(np.mean(err <= 3 * target)),
                   max_abs_z=float(np.abs(z).max()), rms_z=float(np.sqrt(np.mean(z * z))),
                   frac_abs_z_above_3=float(np.mean(np.abs(z) > 3)))
    return out


def entries_at_1e3_device(mc, h, v, idx, pilot: int, target: float = 1e-3, margin: float = 1.2,
                          max_walkers: int = 1 << 26, exact=None):
    """The same two-pass rule with both passes on the device in one call
    (mc_expmv_entries_to_target: the production walker counts are computed on the GPU
    from the pilot, so the host does not wait between the passes).  One pass: no
    re-run of entries that miss the target.  entries_per_s includes the pilot."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    v = h._v(v)
    ti = torch.as_tensor(np.asarray(idx, np.int64), device=dev)
    k = ti.numel()
    est = torch.empty(k, dtype=torch.float64, device=dev)
    se = torch.empty(k, dtype=torch.float64, device=dev)
    nw = torch.empty(k, dtype=torch.int64, device=dev)
    h.entries_to_target(v, ti, pilot, target, margin, 2, max_walkers, est, se, nw)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.entries_to_target(v, ti, pilot, target, margin, 2, max_walkers, est, se, nw)
    seconds = time.perf_counter() - t0
    en, sn, nn = est.cpu().numpy(), se.cpu().numpy(), nw.cpu().numpy()
    rel = sn / np.abs(en)
    out = dict(entries=k, seconds=seconds, entries_per_s_with_pilot=k / seconds,
               pilot_walkers_per_entry=pilot, margin=margin, walkers=int(nn.sum()),
               max_rel_stderr=float(rel.max()), entries_above_target=int((rel > target).sum()),
               final_walkers_max=int(nn.max()))
    if exact is not None:
        ex = np.asarray(exact, np.float64)
        err = np.abs(en - ex) / np.abs(ex)
        z = (en - ex) / np.maximum(sn, 1e-300)
        out.update(achieved_max_rel_err=float(err.max()),
                   achieved_median_rel_err=float(np.median(err)),
                   achieved_frac_within_1e3=float(np.mean(err <= target)),
                   achieved_frac_within_3e3=float(np.mean(err <= 3 * target)),
                   max_abs_z=float(np.abs(z).max()), rms_z=float(np.sqrt(np.mean(z * z))))
    return out


def bench_grid2d_entries(mc, seed):
    """2-D Dirichlet Laplacian 32x32, t = 0.1, 16 entries, FP64: entries/s at 1e-3,
    and the achieved errors against exp(tA) v from expm_multiply."""
    import scipy.sparse.linalg as sla
    from paper_1904_12759_amd import workloads as wl
    w = wl.config_grid2d_entries()
    x = sla.expm_multiply((w.t * w.a.to_scipy()).tocsr(), np.asarray(w.v, np.float64))
    h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed)
    entries_at_1e3(mc, h, w.v, w.idx, 10_000)                       # warm-up
    r = entries_at_1e3(mc, h, w.v, w.idx, 10_000, exact=x[w.idx])
    r["workload"] = "grid2d 32x32 Dirichlet, t=0.1, 16 entries, FP64, two-pass (pilot 1e4)"
    r["device_sized"] = entries_at_1e3_device(mc, h, w.v, w.idx, 10_000, exact=x[w.idx])
    return r


def bench_locality(mc, seed, steps=5):
    """Kernel time of full-vector runs with the rows in input order, relabelled
    hot-first (descending exit rate), relabelled with the hottest rows staged in LDS
    (64-thread blocks staging per block, or 256-thread blocks of which only the
    resident ones are launched, each staging once), relabelled with the wave re-sort
    by current node every 1, 4 or 16 events, and with 64-byte slots.  Workloads: BA
    n=1e5 (the tables stay in cache) at t = 1 and t = 16, and two graphs whose tables
    do not (ER and Chung-Lu power-law, n = 1e6, mean degree 8, A = adjacency /
    lambda_max, FP64, 64 walkers per node) at t = 0.5 and t = 4.  All variants of a
    workload give bitwise identical results."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    dev = torch.device("cuda", torch.cuda.current_device())
    variants = (("input_order", dict()), ("relabel", dict(relabel=1)),
                ("relabel_lds16k_b64", dict(relabel=1, lds_budget=16384)),
                ("relabel_lds16k_b256", dict(relabel=1, lds_budget=16384, walkers_per_block=256)),
                ("relabel_lds64k_b256", dict(relabel=1, lds_budget=65536, walkers_per_block=256)),
                ("relabel_resort1", dict(relabel=1, resort_period=1)),
                ("relabel_resort4", dict(relabel=1, resort_period=4)),
                ("relabel_resort16", dict(relabel=1, resort_period=16)),
                ("slots64B", dict(slot_rows=1)), ("separate_slots", dict(slot_rows=-1)))
    ba = wl.config_ba_full()
    er = wl.er_graph(1_000_000, 8.0, 11)
    er = wl.scaled(er, 1.0 / wl.lambda_max(er))
    cl = wl.chung_lu_graph(1_000_000, 8.0, 2.5, 12)
    cl = wl.scaled(cl, 1.0 / wl.lambda_max(cl))
    cases = (("ba_n1e5_t1", ba.a, 1.0, ba.nwalk, True), ("ba_n1e5_t16", ba.a, 16.0, 100, True),
             ("er_n1e6_t0.5", er, 0.5, 64, False), ("er_n1e6_t4", er, 4.0, 64, False),
             ("cl_n1e6_t0.5", cl, 0.5, 64, False), ("cl_n1e6_t4", cl, 4.0, 64, False))
    out = {}
    for case, a, t, nwalk, fp32 in cases:
        vv = np.random.default_rng(2).random(a.n) if not fp32 else np.ones(a.n)
        v = torch.as_tensor(vv, dtype=torch.float32 if fp32 else torch.float64, device=dev)
        est = torch.empty(a.n, dtype=torch.float64, device=dev)
        se = torch.empty(a.n, dtype=torch.float64, device=dev)
        ref = None
        res = {"nnz": a.nnz, "walkers_per_node": nwalk, "fp32": fp32}
        for name, kw in variants:
            h = mc.MCExpmv(a.rowptr, a.col, a.val, t, seed, fp32=fp32, **kw)
            h.full(v, nwalk, est=est, stderr=se)
            ms = []
            for _ in range(steps):
                h.full(v, nwalk, est=est, stderr=se)
                ms.append(h.stats()["ms"])
            if ref is None:
                ref = est.clone()
                st = h.stats()
                res["events_per_walker"] = st["events"] / st["walkers"]
            res[name] = dict(kernel_ms=float(np.median(ms)), identical=bool(torch.equal(est, ref)))
            del h
        out[case] = res
        log(f"bench: locality {case}: " + ", ".join(
            f"{k} {res[k]['kernel_ms']:.3f}" for k, _ in variants))
    return out


def bench_ba(mc, seed, steps=20):
    """Network communicability: BA n = 1e5, m = 3 (seed 1), A = (0.5/lambda_max)
    adjacency, t = 1, v = 1, full vector with 1000 walkers per node (1e8 walkers),
    FP32 weights: walker-steps/s, the ALU roofline and the gather bytes."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    w = wl.config_ba_full()
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream()
    h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed, fp32=True, stream=stream.cuda_stream)
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    se = torch.empty(w.a.n, dtype=torch.float64, device=dev)
    for _ in range(3):
        h.full(v, w.nwalk, est=est, stderr=se, sync=False)
    h.sync()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        h.full(v, w.nwalk, est=est, stderr=se, sync=False)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h.sync()
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    st = h.stats()
    traffic = measured_traffic(PROFILE_BA)
    lb = gather_bytes_lower_bound(w.a.n, st["jumps"], True)
    rel = (se / est.abs()).cpu().numpy()
    del h
    return dict(workload="BA n=1e5 m=3 seed 1, A=(0.5/lambda_max)*adjacency, t=1, v=1, full "
                         "vector, 1000 walkers/node, EXACT, FP32 weights",
                n=w.a.n, nnz=w.a.nnz, walkers=st["walkers"], events=st["events"],
                jumps=st["jumps"], kernel_ms=kern, ms_per_step=wall * 1e3 / steps,
                walker_steps_per_s=st["events"] / (wall / steps),
                roofline=alu_roofline(st["events"], kern, traffic),
                counters=measured_counters(PROFILE_BA),
                gather_bytes_lower_bound=lb,
                gather_gbs_lower_bound=lb / (kern / 1e3) / 1e9,
                median_rel_stderr=float(np.median(rel)), max_rel_stderr=float(np.max(rel)))


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
                roofline=alu_roofline(st["events"], kern,
                                      measured_traffic(PROFILE_BATCH, KERNEL_SOURCES + [BATCH_SOURCE])),
                hbm_equivalent_frac_no_reuse=achieved / HBM_PEAK_GBS, schedule=b.schedule(),
                traffic=measured_traffic(PROFILE_BATCH, KERNEL_SOURCES + [BATCH_SOURCE]),
                counters=measured_counters(PROFILE_BATCH, KERNEL_SOURCES + [BATCH_SOURCE]),
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


def _exact_moments(a, v, bias, t=1.0):
    """x = exp(tA) v and the exact second moment of the walker value: by Feynman-Kac
    with the jump factors e^{-b}, E[f^2] = exp(tG) v^2 with G_ij = a_ij e^{-b_ij},
    G_ii = 2 d~_i - r~_i (d = r: A has no diagonal)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    deg = np.diff(a.rowptr)
    rows = np.repeat(np.arange(a.n), deg)
    b = np.zeros(a.nnz) if bias is None else np.asarray(bias, np.float64)
    at = a.val * np.exp(b)
    rt = np.bincount(rows, weights=at, minlength=a.n)
    r = np.bincount(rows, weights=a.val, minlength=a.n)
    gm = sp.csr_matrix((a.val * np.exp(-b), a.col, a.rowptr), shape=(a.n, a.n))
    gm = gm + sp.diags(2 * (r + (rt - r)) - rt)
    m2 = sla.expm_multiply((t * gm).tocsr(), v * v)
    x = sla.expm_multiply((t * a.to_scipy()).tocsr(), v)
    return x, m2


def _walkers_to_target(x, m2, idx, target=1e-3):
    """Walkers each entry needs for a relative standard error of `target`, from its
    exact variance."""
    xi = x[idx]
    var = np.maximum(m2[idx] - xi * xi, 0)
    return var / (target * xi) ** 2


def _tail_diagnostics(h, v, nodes, count, proposal):
    """Per start node, from `count` traced walkers: max f / mean f and the effective
    sample size fraction (sum f)^2 / (count sum f^2) of the walker values f (the
    importance-weighted values when the proposal is on)."""
    rat, ess = [], []
    for i in nodes:
        f = h.trace(v, int(i), 0, count, proposal=proposal)[3]
        m = f.mean()
        rat.append(float(f.max() / m))
        ess.append(float(f.sum() ** 2 / (count * (f * f).sum())))
    return dict(nodes=[int(i) for i in nodes], walkers=count, max_over_mean=rat, ess_frac=ess)


def bench_learned(mc, seed, n=1_000_000, m=4, plain_cap=1 << 28):
    """Learned vs plain proposal on BA(n=1e6, m=4), t = 1, 1024 entries (the 256
    highest-degree nodes and 768 uniform ones).  Walker-steps to 1e-3 relative
    standard error for both walks from exact per-entry variances (exact second
    moments; the plain walk's count is analytic); the learned walk's production run at
    1e-3 on all entries with its achieved errors against expm_multiply; and, measured
    side by side, both walks at 1e-3 on the uniform entries the plain walk can reach
    (exact plain walker count <= plain_cap).  The network is trained on the graph of
    seed 1 and also applied, unchanged, to a held-out graph of seed 2."""
    import torch
    t_gen = time.perf_counter()
    a, v, idx, lam = _ba_learned_case(n, m, 1)
    t_gen = time.perf_counter() - t_gen
    deg = np.diff(a.rowptr)
    hubs = np.argsort(-deg)[:256]

    def events_per_walker(h, vv, ii):
        h.entries(vv, ii, 1 << 14)      # plain, or tilted once a proposal is installed
        st = h.stats()
        return st["events"] / st["walkers"]

    log("bench: learned: exact moments (plain)")
    h = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, seed)
    ev_plain = events_per_walker(h, v, idx)
    x, m2p = _exact_moments(a, v, None)
    n_plain = _walkers_to_target(x, m2p, idx)
    # the plain walk at 1e-3, measured, on the uniform entries it can reach
    uni = np.setdiff1d(idx, hubs)
    nu = _walkers_to_target(x, m2p, uni)
    feas = uni[nu <= plain_cap]
    log(f"bench: learned: plain walk at 1e-3 on {len(feas)} uniform entries")
    entries_at_1e3(mc, h, v, feas[:16], 10_000)                       # warm-up
    plain_feas = entries_at_1e3(mc, h, v, feas, 10_000, exact=x[feas])
    diag_nodes = np.concatenate([hubs[:4], feas[:4]])
    tail_plain = _tail_diagnostics(h, v, diag_nodes, 100_000, False)
    log("bench: learned: training the proposal")
    rep = h.learn_proposal(v, pilot_walkers=256, steps=400, batch=1 << 16, lr=3e-3, seed=1)
    bias = h.get_proposal().cpu().numpy()
    ev_learn = events_per_walker(h, v, idx)
    _, m2l = _exact_moments(a, v, bias)
    n_learn = _walkers_to_target(x, m2l, idx)
    steps_p = float(n_plain.sum() * ev_plain)
    steps_l = float(n_learn.sum() * ev_learn)
    prod = entries_at_1e3(mc, h, v, idx, 10_000, exact=x[idx])
    prod["device_sized"] = entries_at_1e3_device(mc, h, v, idx, 10_000, max_walkers=1 << 24,
                                                 exact=x[idx])
    learn_feas = entries_at_1e3(mc, h, v, feas, 10_000, exact=x[feas])
    tail_learn = _tail_diagnostics(h, v, diag_nodes, 100_000, True)
    out = dict(workload=f"BA n={n} m={m} seed 1, A=(0.5/lambda_max)*adjacency "
                        f"(lambda_max={lam:.6g}), t=1, v~U[0,1], {len(idx)} entries "
                        "(256 highest degree + uniform)", generation_s=t_gen,
               walker_steps_to_1e3_plain_exact=steps_p,
               walker_steps_to_1e3_learned_exact=steps_l,
               gain_walker_steps=steps_p / steps_l if steps_l > 0 else None,
               plain_steps_are="analytic: exact per-entry variances (exp(tG) v^2) x measured "
                               "steps per walker",
               events_per_walker_plain=ev_plain, events_per_walker_learned=ev_learn,
               learned_production=prod,
               learned_entries_per_s_at_1e3=prod["entries_per_s"],
               learned_max_rel_stderr=prod["max_rel_stderr"],
               learned_max_rel_err_vs_exact=prod.get("achieved_max_rel_err"),
               measured_side_by_side=dict(
                   entries=f"{len(feas)} of the {len(uni)} uniform entries whose exact plain "
                           f"walker count to 1e-3 is at most {plain_cap}",
                   plain=plain_feas, learned=learn_feas,
                   entries_per_s_ratio=learn_feas["entries_per_s"] / plain_feas["entries_per_s"],
                   walkers_ratio=plain_feas["walkers"] / learn_feas["walkers"]),
               tail_diagnostics=dict(plain=tail_plain, learned=tail_learn),
               train=dict(initial_loss=rep["initial_loss"], final_loss=rep["final_loss"],
                          steps=rep["steps"], pilot_ms=rep["pilot_ms"], train_ms=rep["train_ms"]))
    del h
    # held-out graph: same network, features of the new graph
    log("bench: learned: held-out graph")
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
    x2, m2p2 = _exact_moments(a2, v2, None)
    _, m2l2 = _exact_moments(a2, v2, bias2.cpu().numpy())
    steps_p2 = float(_walkers_to_target(x2, m2p2, idx2).sum() * ev_plain2)
    steps_l2 = float(_walkers_to_target(x2, m2l2, idx2).sum() * ev_learn2)
    prod2 = entries_at_1e3(mc, h2, v2, idx2, 10_000, exact=x2[idx2])
    out["held_out"] = dict(
        workload=f"BA n={n} m={m} seed 2 (lambda_max={lam2:.6g}), same recipe; network "
                 "trained on seed 1, not retrained",
        walker_steps_to_1e3_plain_exact=steps_p2, walker_steps_to_1e3_learned_exact=steps_l2,
        gain_walker_steps=steps_p2 / steps_l2 if steps_l2 > 0 else None,
        learned_production=prod2,
        learned_entries_per_s_at_1e3=prod2["entries_per_s"],
        learned_max_rel_stderr=prod2["max_rel_stderr"],
        learned_max_rel_err_vs_exact=prod2.get("achieved_max_rel_err"))
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
        kms = float(np.median(ms))
        out[name] = dict(ms_per_tc=kms, first_call_s=first, tc=tc,
                         tc_n=tc / a.n, rel_stderr=tse / abs(tc),
                         rel_err_vs_exact=(tc - exact) / exact,
                         events=st["events"], jumps=st["jumps"],
                         walker_steps_per_s=st["events"] / (kms / 1e3),
                         # the call is bound by random gathers, not arithmetic: the ALU
                         # fraction beside the gather bytes (no reuse) per second
                         roofline=alu_roofline(st["events"], kms, None),
                         gather_gbs_no_reuse=st["alg_bytes"] / (kms / 1e3) / 1e9)
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


def bench_qmc(mc, seed, seeds=8):
    """The randomised-lattice first event (opts.qmc_first) against the plain walk:
    entries/s at 1e-3 on the grid2d 32x32 entries workload (FP64; the lattice's
    standard error from its replicate means), and on the BA n=1e5 full vector (1000
    walkers per node, FP32) the per-node variance of the estimates over independent
    seeds, with the kernel times."""
    import scipy.sparse.linalg as sla
    import torch
    from paper_1904_12759_amd import workloads as wl
    out = {}
    g2 = wl.config_grid2d_entries()
    x = sla.expm_multiply((g2.t * g2.a.to_scipy()).tocsr(), np.asarray(g2.v, np.float64))
    # the lattice's pilot: 32 replicates of 512, whose replicate standard error (31
    # degrees of freedom, about 13 % relative error) sizes the production run, so its
    # margin covers 2.5 such errors, (1 + 2.5 / sqrt(62))^2 = 1.73, for one pass; and
    # every production entry gets at least 16 replicates, since with one replicate
    # the reported error falls back to the i.i.d. formula, which overstates it
    for name, q, pilot, margin, floor in (("plain", False, 10_000, 1.2, 2),
                                          ("lattice", True, 32 * 512, 1.73, 16 * 512)):
        h = mc.MCExpmv(g2.a.rowptr, g2.a.col, g2.a.val, g2.t, seed, qmc=q)
        entries_at_1e3(mc, h, g2.v, g2.idx, pilot, margin=margin, min_walkers=floor)
        r = entries_at_1e3(mc, h, g2.v, g2.idx, pilot, margin=margin, min_walkers=floor,
                           exact=x[g2.idx])
        r["margin"] = margin
        r["min_walkers"] = floor
        out[f"grid2d_entries_at_1e3_{name}"] = r
    w = wl.config_ba_full()
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    res = {}
    for name, q in (("plain", False), ("lattice", True)):
        ests, ms = [], []
        for k in range(seeds):
            h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed + k, fp32=True, qmc=q)
            e, _ = h.full(v, w.nwalk)
            e, _ = h.full(v, w.nwalk)
            ms.append(h.stats()["ms"])
            ests.append(e.cpu().numpy())
            del h
        res[name] = (np.var(np.array(ests), axis=0, ddof=1), float(np.median(ms)))
    gain = res["plain"][0] / np.maximum(res["lattice"][0], 1e-300)
    deg = np.diff(w.a.rowptr)
    out["ba_full"] = dict(
        workload=f"BA n=1e5 m=3, full vector, 1000 walkers/node, FP32; variance over {seeds} seeds",
        kernel_ms_plain=res["plain"][1], kernel_ms_lattice=res["lattice"][1],
        median_variance_gain=float(np.median(gain)),
        median_variance_gain_degree_3=float(np.median(gain[deg == 3])),
        median_variance_gain_top_1pct_degree=float(np.median(gain[deg >= np.quantile(deg, 0.99)])),
        total_variance_gain=float(res["plain"][0].sum() / res["lattice"][0].sum()))
    # the headline workload: kernel time and per-node variance over seeds
    w = wl.config_grid3d_full(256)
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    res = {}
    for name, q in (("plain", False), ("lattice", True)):
        ests, ms = [], []
        for k in range(4):
            h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed + k, fp32=True, qmc=q)
            e, _ = h.full(v, w.nwalk)
            e, _ = h.full(v, w.nwalk)
            ms.append(h.stats()["ms"])
            ests.append(e.cpu().numpy())
            del h, e
        res[name] = (np.var(np.array(ests), axis=0, ddof=1), float(np.median(ms)))
    gain = res["plain"][0] / np.maximum(res["lattice"][0], 1e-300)
    out["grid3d_full"] = dict(
        workload="grid3d 256^3 (the headline workload), full vector, 256 walkers/node, FP32; "
                 "variance over 4 seeds",
        kernel_ms_plain=res["plain"][1], kernel_ms_lattice=res["lattice"][1],
        median_variance_gain=float(np.median(gain)),
        total_variance_gain=float(res["plain"][0].sum() / res["lattice"][0].sum()))
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


def bench_stencil(mc, seed, steps=5):
    """The matrix-free 7-point walk (mc_expmv_create_stencil7) against the table walk
    on the headline grid3d 256^3 workload (t = 0.05, 256 walkers per node, EXACT,
    FP32 weights): kernel time, walker-steps/s, device bytes of the operator, and
    the two estimates' agreement (both unbiased; different jump rules, so not
    bitwise equal): the rms over nodes of their difference in units of the
    combined standard error."""
    import torch
    from paper_1904_12759_amd import workloads as wl
    w = wl.config_grid3d_full(256)
    m = 256
    dev = torch.device("cuda", torch.cuda.current_device())
    v = torch.as_tensor(w.v, dtype=torch.float32, device=dev)
    fx, fy, fz, diag = wl.stencil7_faces(w.a, m, m, m)
    res = {}
    for name in ("table", "stencil"):
        if name == "table":
            h = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, seed, fp32=True)
        else:
            h = mc.MCExpmv.stencil7(m, m, m, fx, fy, fz, diag, w.t, seed, fp32=True)
        est = torch.empty(w.a.n, dtype=torch.float64, device=dev)
        se = torch.empty(w.a.n, dtype=torch.float64, device=dev)
        h.full(v, w.nwalk, est=est, stderr=se)
        ms = []
        for _ in range(steps):
            h.full(v, w.nwalk, est=est, stderr=se)
            ms.append(h.stats()["ms"])
        st = h.stats()
        kms = float(np.median(ms))
        res[name] = dict(kernel_ms=kms, walker_steps_per_s=st["events"] / (kms / 1e3),
                         events=st["events"], jumps=st["jumps"],
                         roofline=alu_roofline(st["events"], kms, None))
        res[name + "_est"] = (est, se)
        del h
    (e1, s1), (e2, s2) = res.pop("table_est"), res.pop("stencil_est")
    d2 = s1 * s1 + s2 * s2
    pos = d2 > 0
    z = ((e1 - e2)[pos] / torch.sqrt(d2[pos])).cpu().numpy()
    res["workload"] = "grid3d 256^3 (the headline workload), full vector, 256 walkers/node, FP32"
    res["speedup"] = res["table"]["kernel_ms"] / res["stencil"]["kernel_ms"]
    # device bytes of the operator: a 32 B state record and d in both precisions (12 B)
    # per node; the tables hold a 16 B row record, d, r (8 B) per node and a 16 B slot
    # per CSR position
    res["operator_bytes_stencil"] = (32 + 12) * w.a.n
    res["operator_bytes_table"] = (16 + 12 + 8) * w.a.n + 16 * w.a.nnz
    res["rms_z_table_vs_stencil"] = float(np.sqrt(np.mean(z * z)))
    res["frac_abs_z_above_4"] = float(np.mean(np.abs(z) > 4))
    return res


def run_extras(mc, wl, args, out):
    names = ["ba", "locality", "entries", "learned", "batched", "forward", "cond", "qmc",
             "splitting", "isim", "stencil"]
    extras = [] if args.no_extras or args.extras == "none" else \
        names if args.extras == "all" else [x for x in args.extras.split(",") if x]
    unknown = [x for x in extras if x not in names]
    if unknown:
        print(f"bench.py: unknown extras {unknown}; choose from {names}", file=sys.stderr)
        sys.exit(2)
    if "ba" in extras:
        log("bench: BA n=1e5 full vector")
        out["ba_n1e5"] = bench_ba(mc, args.seed)
    if "locality" in extras:
        log("bench: locality variants")
        out["locality"] = bench_locality(mc, args.seed)
    if "entries" in extras:
        log("bench: entries/s at 1e-3 (grid2d)")
        out["entries_at_1e3"] = bench_grid2d_entries(mc, args.seed)
    if "learned" in extras:
        log("bench: learned vs plain (BA n=1e6 m=4)")
        out["learned_vs_plain"] = bench_learned(mc, args.seed)
    if "batched" in extras:
        log("bench: batched 64 instances")
        out["batched_64"] = bench_batched(mc, args.seed)
    if "forward" in extras:
        log("bench: forward total communicability (small world n=1e6)")
        out["forward_tc"] = bench_forward_tc(mc, args.seed)
    if "cond" in extras:
        log("bench: first-jump conditioning vs plain")
        out["conditioning"] = bench_conditioning(mc, args.seed)
    if "qmc" in extras:
        log("bench: randomised-lattice first event vs plain")
        out["qmc"] = bench_qmc(mc, args.seed)
    if "splitting" in extras:
        log("bench: splitting study (small world n=100, 1000)")
        out["splitting"] = bench_splitting(mc, args.seed)
    if "isim" in extras:
        log("bench: ranking study (small world n=1000, 10000)")
        out["isim"] = bench_isim(mc, args.seed)
    if "stencil" in extras:
        log("bench: matrix-free stencil walk vs table walk (grid3d 256^3)")
        out["stencil"] = bench_stencil(mc, args.seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the headline's error against expm_multiply (about 20 s of CPU)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every extra measurement (same as --extras none)")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extra measurements after the main step: "
                         "ba, locality, entries, learned, batched, forward, cond, qmc, "
                         "splitting, isim; 'all' or 'none'")
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the extras (for profiling them on their own)")
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
    if args.skip_headline:
        out = {"metric": METRIC, "note": "extras only (--skip-headline)"}
        run_extras(mc, wl, args, out)
        print(json.dumps(out), flush=True)
        return
    log("bench: building workload (grid3d 256^3)")
    t0 = time.perf_counter()
    w = wl.config_grid3d_full(256)
    gen_s = time.perf_counter() - t0
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

    log(f"bench: timing {args.steps} steps")
    # HIP events on the stream the walk is launched on bracket each launch
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
    traffic = measured_traffic()
    lb = gather_bytes_lower_bound(w.a.n, st["jumps"], True)
    e_np = est.cpu().numpy()
    s_np = se.cpu().numpy()
    rel = s_np / np.abs(e_np)
    del h

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
            "workload": "grid3d 256^3 variable-coefficient diffusion (7-point, kappa log-uniform "
                        "[0.1,10], harmonic faces, Dirichlet), t=0.05, v = bump + U[0,1], full "
                        "vector exp(tA)v, 256 walkers/node, EXACT weights, FP32 weights",
            "n": w.a.n, "nnz": w.a.nnz, "walkers": st["walkers"], "events_per_step": events,
            "jumps_per_step": st["jumps"],
        },
        "walkers_per_s": st["walkers"] / (ms_per_step / 1e3),
        "kernel_ms": kern_ms,
        "setup_ms": setup_s * 1e3,
        "generation_s": gen_s,
        "median_rel_stderr": float(np.median(rel)),
        "max_rel_stderr": float(np.max(rel)),
        "roofline": alu_roofline(events, kern_ms, traffic),
        # the committed profile's counters: what the VALU is busy with, occupancy, L2
        "counters": measured_counters(),
        # gathers the walk must make (no reuse between entries), as a bandwidth: a
        # work-equivalent figure, not HBM use (which is roofline.traffic)
        "gather_bytes_lower_bound": lb,
        "gather_gbs_lower_bound": lb / (kern_ms / 1e3) / 1e9,
    }
    if not args.no_accuracy:
        log("bench: headline error against expm_multiply")
        import scipy.sparse.linalg as sla
        x = sla.expm_multiply((w.t * w.a.to_scipy()).tocsr(), np.asarray(w.v, np.float64))
        err = np.abs(e_np - x) / np.abs(x)
        # entries whose 256 walkers all stayed have a zero standard error (and the
        # estimate e^{td} v of a walker that never moves): z only where se > 0
        pos = s_np > 0
        z = (e_np[pos] - x[pos]) / s_np[pos]
        out["accuracy"] = dict(median_rel_err=float(np.median(err)),
                               p99_rel_err=float(np.quantile(err, 0.99)),
                               max_rel_err=float(err.max()),
                               entries_with_zero_stderr=int((~pos).sum()),
                               rms_z=float(np.sqrt(np.mean(z * z))),
                               frac_abs_z_above_3=float(np.mean(np.abs(z) > 3)),
                               reference="scipy expm_multiply, FP64")
    run_extras(mc, wl, args, out)
    if not args.no_cpu:
        log("bench: CPU oracle baseline (grid3d samples)")
        try:
            nthreads = len(os.sched_getaffinity(0))
        except AttributeError:
            nthreads = os.cpu_count() or 1
        out["cpu_baseline"] = cpu_baseline(w, args.seed, nthreads, events)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
