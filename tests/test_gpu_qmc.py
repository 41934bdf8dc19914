"""GPU parity of the randomised-lattice first event (opts.qmc_first) against the
oracle's own transcription: per-walker final states, events and jumps
bit-identical, per-walker values and estimates within 1e-12 (FP64) / 1e-5 (FP32),
replicate standard errors within 1e-8; the option leaves later events and the
plain walk alone; the lattice estimate is unbiased against dense expm."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle
import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl
import refs

pytestmark = pytest.mark.gpu


def _v_for(v, fp32):
    return np.asarray(v, np.float32).astype(np.float64) if fp32 else np.asarray(v, np.float64)


def _close(a, b, rtol):
    a, b = np.asarray(a), np.asarray(b)
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1e-300))


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("mode", [mc.EXACT, mc.STRANG])
def test_lattice_paths_and_estimates_match_oracle(fp32, mode):
    a = wl.grid2d(20)
    v = np.random.default_rng(4).uniform(0.2, 1.0, a.n)
    t = 0.35
    bits = 10 if fp32 else 9
    g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 91, mode=mode, dt=t / 5, fp32=fp32, qmc=True)
    o = Oracle(a.rowptr, a.col, a.val, t, 91, mode=mode, dt=t / 5, qmc=True, qmc_bits=bits)
    vo = _v_for(v, fp32)
    tol = 1e-5 if fp32 else 1e-12
    for start, w0, cnt in ((0, 0, 3000), (57, 0, 2048), (399, 100, 1500)):
        xg, evg, jug, fg = g.trace(v, start, w0, cnt)
        xo, evo, juo, fo, _ = o.trace(vo, start, w0, cnt)
        assert np.array_equal(xg, xo) and np.array_equal(evg, evo) and np.array_equal(jug, juo)
        assert _close(fg, fo, tol)
    idx = np.array([0, 5, 57, 200, 399, 57], np.int64)
    for m in (256, 700, 4096, 5 * 1024 + 37):             # part of one, one and several replicates, ragged
        est, se = g.entries(v, idx, m)
        eo, so = o.estimate(vo, idx, m, threads=4)
        assert _close(est.cpu().numpy(), eo, tol), m
        assert _close(se.cpu().numpy(), so, 1e-5 if fp32 else 1e-8), m
    # full vector equals entries, and the production path (own walker counts)
    est, se = g.full(v, 2048)
    ee, es = g.entries(v, np.arange(a.n), 2048)
    assert torch.equal(est, ee) and torch.equal(se, es)
    counts = np.array([600, 3000, 5000, 1024, 2100, 9000], np.int64)
    em, sm = g.entries_multi(v, idx, counts)
    for i, m in enumerate(counts):
        e1, s1 = g.entries(v, idx[i:i + 1], int(m))
        assert torch.equal(em[i:i + 1], e1) and torch.equal(sm[i:i + 1], s1)


def test_lattice_off_is_the_plain_walk_and_rejects_conditioning():
    a = wl.grid2d(12)
    v = np.random.default_rng(1).random(a.n)
    p = mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 7)
    q = mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 7, qmc=False)
    assert torch.equal(p.full(v, 1000)[0], q.full(v, 1000)[0])
    with pytest.raises(mc.MCError):
        mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 7, qmc=True, cond=True)
    with pytest.raises(mc.MCError):
        mc.MCExpmv(a.rowptr, a.col, a.val, 0.4, 7, qmc=True, relabel=1)


def test_lattice_unbiased_against_dense_expm():
    n = 30
    dense = refs.random_metzler(n, 0.2, 61, symmetric=False)
    a = wl.from_dense(dense)
    t = 0.7
    v = np.random.default_rng(62).uniform(0.2, 1.0, n)
    ref = refs.expm_v(dense, t, v)
    zs = []
    for seed in range(24):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 3000 + seed, qmc=True)
        est, se = g.full(v, 16 * 512)
        zs.append((est.cpu().numpy() - ref) / se.cpu().numpy())
    z = np.array(zs)
    # 16 replicate means per estimate: Student's t with 15 degrees of freedom
    assert abs(z.mean()) < 4.5 * np.sqrt(15 / 13 / z.size)
    assert abs(np.mean(z * z) - 15 / 13) < 0.25


def test_lattice_full_size_sampled_parity():
    """The headline workload (grid3d 256^3, full vector, 256 walkers per node: a quarter
    of a 1024-walker replicate, FP32) with the lattice first event, in the launch
    configuration the benchmark times: sampled nodes against the oracle's lattice walk
    (estimates within 1e-5; one partial replicate, so the i.i.d. standard error)."""
    w = wl.config_grid3d_full(256)
    g = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, fp32=True, qmc=True)
    est, se = g.full(w.v, w.nwalk)
    est, se = est.cpu().numpy(), se.cpu().numpy()
    assert np.isfinite(est).all()
    rng = np.random.default_rng(2)
    sample = np.unique(np.concatenate([[0, w.a.n - 1], rng.choice(w.a.n, 300, replace=False)]))
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, qmc=True, qmc_bits=10)
    eo, so = o.estimate(_v_for(w.v, True), sample, w.nwalk, threads=8)
    assert _close(est[sample], eo, 1e-5)
    assert _close(se[sample], so, 1e-5)
