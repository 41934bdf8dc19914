"""GPU tests of the batched launch (persistent kernel, graph replay, autotuner).

Each instance of a batch must give exactly (bitwise) what a separate handle
with the same settings and instance id gives, whatever the schedule, and agree
with the CPU oracle to the single-instance tolerances.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle
import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl
import refs

pytestmark = pytest.mark.gpu


def _mixed_instances():
    rng = np.random.default_rng(11)
    out = []
    mats = [wl.grid2d(12), wl.from_dense(refs.random_metzler(40, 0.2, 1, False)),
            wl.cycle_graph(25, 0.9), wl.er_graph(3000, 8.0, 5),
            wl.from_dense(refs.random_metzler(30, 0.3, 2, True))]
    specs = [  # (matrix, t, mode, fp32, entries?, walkers)
        (0, 0.4, mc.EXACT, False, True, 2500),
        (1, 0.9, mc.STRANG, False, False, 300),
        (2, 1.3, mc.LIE, True, True, 1024),
        (3, 0.5, mc.EXACT, True, False, 64),
        (4, 0.7, mc.EXACT, False, True, 5000),
        (0, 0.2, mc.LIE, False, False, 1500),
    ]
    for i, (mi, t, mode, fp32, entries, nw) in enumerate(specs):
        a = mats[mi]
        v = rng.uniform(0.1, 1.0, a.n)
        d = dict(rowptr=a.rowptr, col=a.col, val=a.val, t=t, v=v, mode=mode, dt=0.05,
                 fp32=fp32, n_walkers=nw, instance_id=100 + i)
        if entries:
            d["idx"] = rng.choice(a.n, 9, replace=True).astype(np.int64)
        out.append((d, a))
    return out


INSTANCES = _mixed_instances()


def _separate(d, a, seed):
    g = mc.MCExpmv(a.rowptr, a.col, a.val, d["t"], seed, mode=d["mode"], dt=d["dt"],
                   fp32=d["fp32"], instance=d["instance_id"])
    if "idx" in d:
        return g.entries(d["v"], d["idx"], d["n_walkers"])
    return g.full(d["v"], d["n_walkers"])


def test_batch_equals_separate_handles():
    seed = 99
    b = mc.MCBatch([d for d, _ in INSTANCES], seed, walkers_per_block=256, blocks_per_cu=4)
    est, se = b.run()
    for i, (d, a) in enumerate(INSTANCES):
        e1, s1 = _separate(d, a, seed)
        assert torch.equal(est[i], e1), i
        assert torch.equal(se[i], s1), i
    st = b.stats()
    assert st["events"] == st["walkers"] + st["jumps"]


def test_batch_finalize_groups_of_several_waves():
    """Instances whose entries span up to 4395 chunks (merged by 256 or 1024 lanes, so
    across the waves of a block), between instances with one chunk and a few: every
    instance bitwise equal to a separate handle."""
    rng = np.random.default_rng(5)
    a = wl.from_dense(refs.random_metzler(40, 0.2, 1, False))
    specs = [(False, 1000, 3), (True, 70_000, 5), (False, 2_250_000, 2), (True, 300, 4),
             (True, 4_500_000, 1), (False, 600_000, 3), (False, 9000, 2)]
    inst = []
    for i, (fp32, nw, k) in enumerate(specs):
        inst.append(dict(rowptr=a.rowptr, col=a.col, val=a.val, t=0.6, v=rng.uniform(0.1, 1.0, a.n),
                         mode=mc.EXACT, dt=0.05, fp32=fp32, n_walkers=nw, instance_id=300 + i,
                         idx=rng.choice(a.n, k, replace=True).astype(np.int64)))
    seed = 4
    est, se = mc.MCBatch(inst, seed).run()
    for i, d in enumerate(inst):
        e1, s1 = _separate(d, a, seed)
        assert torch.equal(est[i], e1), i
        assert torch.equal(se[i], s1), i


def test_batch_with_slot_rows_equals_separate_handles():
    """Every instance with 64-byte slots (slot_rows=1 for the batch) bitwise equal to a
    separate handle with the separate tables."""
    seed = 99
    est, se = mc.MCBatch([d for d, _ in INSTANCES], seed, slot_rows=1).run()
    for i, (d, a) in enumerate(INSTANCES):
        e1, s1 = _separate(d, a, seed)
        assert torch.equal(est[i], e1), i
        assert torch.equal(se[i], s1), i


def test_batch_schedule_and_replay_do_not_change_results():
    b = mc.MCBatch([d for d, _ in INSTANCES], 7, walkers_per_block=128, blocks_per_cu=2)
    ref = [e.clone() for e in b.run()[0]]
    refs_se = [s.clone() for s in b.stderr]
    for wpb, bpc, grp in [(256, 8, 0), (256, 4, 16), (64, 16, 1), (128, 8, 128)]:
        b.set_schedule(wpb, bpc, grp)
        for rep in range(3):
            for e in b.est:
                e.fill_(-1.0)
            torch.cuda.synchronize()
            x = torch.randn(1000, device="cuda").sum()       # unrelated eager work between replays
            b.run()
            for i in range(len(ref)):
                assert torch.equal(b.est[i], ref[i]), (wpb, bpc, grp, rep, i)
                assert torch.equal(b.stderr[i], refs_se[i])
            del x


def test_batch_without_graph_matches():
    b1 = mc.MCBatch([d for d, _ in INSTANCES], 5, walkers_per_block=256, blocks_per_cu=4)
    b2 = mc.MCBatch([d for d, _ in INSTANCES], 5, walkers_per_block=256, blocks_per_cu=4,
                    use_graph=False)
    e1, _ = b1.run()
    e2, _ = b2.run()
    for x, y in zip(e1, e2):
        assert torch.equal(x, y)


def test_batch_matches_oracle():
    seed = 3
    b = mc.MCBatch([d for d, _ in INSTANCES], seed, walkers_per_block=256, blocks_per_cu=4)
    est, _ = b.run()
    for i, (d, a) in enumerate(INSTANCES):
        if a.n > 1000:
            continue
        o = Oracle(a.rowptr, a.col, a.val, d["t"], seed, mode=d["mode"], dt=d["dt"],
                   instance=d["instance_id"])
        v = np.asarray(d["v"], np.float32).astype(np.float64) if d["fp32"] else d["v"]
        eo, _ = o.estimate(v, d.get("idx"), d["n_walkers"])
        tol = 1e-5 if d["fp32"] else 1e-12
        got = est[i].cpu().numpy()
        assert np.all(np.abs(got - eo) <= tol * np.abs(eo)), i


def test_autotune_picks_a_schedule_and_caches_it(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MC_EXPMV_TUNE_CACHE", str(cache))
    insts = [d for d, _ in INSTANCES]
    b = mc.MCBatch(insts, 1)
    sc = b.schedule()
    assert sc["walkers_per_block"] in (64, 128, 256) and sc["blocks_per_cu"] >= 1
    assert cache.exists() and cache.read_text().strip()
    e1 = [e.clone() for e in b.run()[0]]
    b2 = mc.MCBatch(insts, 1)                  # served from the cache
    assert b2.schedule() == sc
    e2, _ = b2.run()
    for x, y in zip(e1, e2):
        assert torch.equal(x, y)


def test_batch_out_of_range_entry_is_reported():
    d, a = INSTANCES[0]
    bad = dict(d)
    bad["idx"] = np.array([0, a.n + 5], np.int64)
    b = mc.MCBatch([bad, INSTANCES[1][0]], 1, walkers_per_block=256, blocks_per_cu=2)
    with pytest.raises(mc.MCError) as ei:
        b.run()
    assert ei.value.code == 4


def test_batched_config_scaled_down():
    """The 64-instance ER / power-law mix (n up to 3e4 here), sampled oracle parity."""
    ws = wl.batched_instances(count=64, nmax=3e4)
    insts = [dict(rowptr=w.a.rowptr, col=w.a.col, val=w.a.val, t=w.t, v=w.v, idx=w.idx,
                  n_walkers=w.nwalk, instance_id=k) for k, w in enumerate(ws)]
    b = mc.MCBatch(insts, 12759)
    est, se = b.run()
    st = b.stats()
    assert st["walkers"] == sum((len(w.idx) if w.idx is not None else w.a.n) * w.nwalk
                                for w in ws)
    for k in (0, 1, 2, 3, 17, 62):
        w = ws[k]
        o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, instance=k)
        if w.idx is not None:
            eo, _ = o.estimate(w.v, w.idx, w.nwalk, threads=8)
            got = est[k].cpu().numpy()
        else:
            sample = np.arange(0, w.a.n, max(1, w.a.n // 50))
            eo, _ = o.estimate(w.v, sample, w.nwalk, threads=8)
            got = est[k].cpu().numpy()[sample]
        assert np.all(np.abs(got - eo) <= 1e-12 * np.abs(eo)), k


def test_batched_config_full_size_sampled():
    """The benchmark's 64-instance set at full size (n log-uniform up to 1e6), schedule
    from the autotuner as the benchmark runs it: sampled oracle parity on instances of
    every type, among them the largest of each kind."""
    ws = wl.batched_instances(count=64)
    insts = [dict(rowptr=w.a.rowptr, col=w.a.col, val=w.a.val, t=w.t, v=w.v, idx=w.idx,
                  n_walkers=w.nwalk, instance_id=k) for k, w in enumerate(ws)]
    os.environ.pop("MC_EXPMV_TUNE_CACHE", None)
    b = mc.MCBatch(insts, 12759)
    est, se = b.run()
    sizes = np.array([w.a.n for w in ws])
    picks = {0, 1, 2, 3}
    for kind in range(4):
        ks = [k for k in range(64) if k % 4 == kind]
        picks.add(max(ks, key=lambda k: sizes[k]))
    for k in sorted(picks):
        w = ws[k]
        o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, instance=k)
        if w.idx is not None:
            eo, _ = o.estimate(w.v, w.idx, w.nwalk, threads=8)
            got = est[k].cpu().numpy()
        else:
            sample = np.linspace(0, w.a.n - 1, 40).astype(np.int64)
            eo, _ = o.estimate(w.v, sample, w.nwalk, threads=8)
            got = est[k].cpu().numpy()[sample]
        assert np.all(np.abs(got - eo) <= 1e-12 * np.abs(eo)), (k, int(sizes[k]))
