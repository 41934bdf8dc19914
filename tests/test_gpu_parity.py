"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Same seeded inputs on both sides.  Integer results (tables, final states, event
and jump counts) must be bit-identical; estimates must agree within 1e-12
relative in FP64 weight mode and 1e-5 relative in FP32 weight mode (the
oracle is always FP64).  Standard errors agree to 1e-8 relative in FP64: the
GPU forms them from shifted one-pass sums, the oracle with two passes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from oracle import Oracle
import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl
import refs

pytestmark = pytest.mark.gpu

RTOL64 = 1e-12
RTOL32 = 1e-5


def _pair(a: wl.CSR, t, seed, mode=mc.EXACT, dt=0.03125, fp32=False, instance=0,
          max_events=0, **kw):
    g = mc.MCExpmv(a.rowptr, a.col, a.val, t, seed, mode=mode, dt=dt, fp32=fp32,
                   instance=instance, max_events=max_events, **kw)
    o = Oracle(a.rowptr, a.col, a.val, t, seed, mode=mode, dt=dt, instance=instance,
               max_events=max_events)
    return g, o


def _v_for(v, fp32):
    """The vector as the GPU sees it (float32 in FP32 mode), widened for the oracle."""
    return np.asarray(v, np.float32).astype(np.float64) if fp32 else np.asarray(v, np.float64)


def _close(a, b, rtol):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = np.maximum(np.abs(b), 1e-300)
    return np.all(np.abs(a - b) <= rtol * scale)


def _matrices():
    out = {}
    out["sym48"] = wl.from_dense(refs.random_metzler(48, 0.15, 1, True))
    out["nonsym48"] = wl.from_dense(refs.random_metzler(48, 0.2, 2, False, off_scale=2.0))
    a = refs.random_metzler(40, 0.3, 3, False)
    a[5, :] = 0.0
    a[5, 5] = -0.5            # a row with no jumps
    a[7, :] = 0.0
    a[7, [2, 9, 30]] = 0.75    # a uniform row
    out["special40"] = wl.from_dense(a)
    out["grid2d_16"] = wl.grid2d(16)
    out["cycle31"] = wl.cycle_graph(31, 0.8)
    return out


MATS = _matrices()


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("name", sorted(MATS))
def test_tables_bit_identical(name):
    a = MATS[name]
    g, o = _pair(a, 1.0, 5)
    tg, to = g.tables(), o.tables()
    for key in ("r", "d", "inv_r", "deg", "begin", "col", "thr", "alias"):
        assert np.array_equal(tg[key], to[key]), key


def test_tables_bit_identical_ba_config():
    w = wl.config_ba_full(n=20_000)
    g, o = _pair(w.a, w.t, 1)
    tg, to = g.tables(), o.tables()
    for key in ("r", "d", "inv_r", "deg", "begin", "col", "thr", "alias"):
        assert np.array_equal(tg[key], to[key]), key


# ---------------------------------------------------------- walker paths
@pytest.mark.parametrize("mode", [mc.EXACT, mc.STRANG, mc.LIE])
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("name", ["nonsym48", "special40", "grid2d_16"])
def test_paths_bit_identical(name, mode, fp32):
    a = MATS[name]
    t = 1.3
    g, o = _pair(a, t, 777, mode=mode, dt=0.1, fp32=fp32)
    v = np.random.default_rng(4).uniform(0.1, 2.0, a.n)
    vv = _v_for(v, fp32)
    for start in (0, 5, 7, a.n - 1):
        count = 3000
        xg, eg, jg, fg = g.trace(v, start, 10, count)
        xo, eo, jo, fo, _ = o.trace(vv, start, 10, count)
        assert np.array_equal(xg, xo)
        assert np.array_equal(eg, eo)
        assert np.array_equal(jg, jo)
        assert _close(fg, fo, RTOL32 if fp32 else RTOL64)


# ------------------------------------------------------------- estimates
@pytest.mark.parametrize("mode", [mc.EXACT, mc.STRANG, mc.LIE])
@pytest.mark.parametrize("name", sorted(MATS))
def test_entries_match_oracle_fp64(name, mode):
    a = MATS[name]
    t = 0.9
    g, o = _pair(a, t, 4242, mode=mode, dt=0.07)
    v = np.random.default_rng(9).uniform(-1.0, 2.0, a.n)
    idx = np.array([0, 3, 5, 7, a.n - 1, 3, 11], np.int64)
    # 2500 walkers: three chunks, the last one ragged
    est, se = g.entries(v, idx, 2500)
    eo, so = o.estimate(v, idx, 2500)
    assert _close(est.cpu().numpy(), eo, RTOL64)
    assert np.allclose(se.cpu().numpy(), so, rtol=1e-8, atol=1e-300)
    assert est[1].item() == est[5].item()       # duplicate entries are identical


@pytest.mark.parametrize("name", ["sym48", "special40", "grid2d_16"])
def test_full_matches_oracle_and_entries(name):
    a = MATS[name]
    g, o = _pair(a, 0.7, 31)
    v = np.random.default_rng(1).random(a.n)
    est, se = g.full(v, 700)
    eo, so = o.estimate(v, None, 700)
    assert _close(est.cpu().numpy(), eo, RTOL64)
    assert np.allclose(se.cpu().numpy(), so, rtol=1e-8, atol=1e-300)
    idx = np.arange(a.n)[::3]
    e2, s2 = g.entries(v, idx, 700)
    assert torch.equal(e2, est[torch.as_tensor(idx, device=est.device)])
    assert torch.equal(s2, se[torch.as_tensor(idx, device=se.device)])


@pytest.mark.parametrize("mode", [mc.EXACT, mc.STRANG])
def test_fp32_weights_match_oracle(mode):
    a = MATS["nonsym48"]
    g, o = _pair(a, 1.1, 8, mode=mode, dt=0.05, fp32=True)
    v = np.random.default_rng(2).uniform(0.2, 1.0, a.n)
    est, se = g.full(v, 3000)
    eo, so = o.estimate(_v_for(v, True), None, 3000)
    assert _close(est.cpu().numpy(), eo, RTOL32)


def test_results_are_deterministic_and_launch_independent():
    a = MATS["grid2d_16"]
    v = np.random.default_rng(3).random(a.n)
    outs = []
    for block in (64, 128, 256):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 99, walkers_per_block=block)
        outs.append(g.full(v, 1500))
    for e, s in outs[1:]:
        assert torch.equal(e, outs[0][0]) and torch.equal(s, outs[0][1])


def test_instance_id_matches_oracle():
    a = MATS["sym48"]
    g, o = _pair(a, 1.0, 5, instance=17)
    v = np.ones(a.n)
    est, _ = g.entries(v, [1, 2, 3], 4000)
    eo, _ = o.estimate(v, [1, 2, 3], 4000)
    assert _close(est.cpu().numpy(), eo, RTOL64)
    g0 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 5)
    e0, _ = g0.entries(v, [1, 2, 3], 4000)
    assert not torch.equal(e0, est)


# ------------------------------------------------------------ edge cases
def test_t_zero_returns_v():
    a = MATS["nonsym48"]
    v = np.random.default_rng(5).random(a.n)
    for mode in (mc.EXACT, mc.STRANG, mc.LIE):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 0.0, 1, mode=mode, dt=0.1)
        est, se = g.full(v, 64)
        assert np.allclose(est.cpu().numpy(), v, rtol=1e-15, atol=0)
        assert np.all(se.cpu().numpy() <= 1e-15 * v)


def test_single_walker_and_empty_requests():
    a = MATS["sym48"]
    g, o = _pair(a, 1.0, 3)
    v = np.random.default_rng(6).random(a.n)
    est, se = g.entries(v, [4], 1)
    eo, _ = o.estimate(v, [4], 1)
    assert _close(est.cpu().numpy(), eo, RTOL64) and se.item() == 0.0
    est, se = g.entries(v, np.zeros(0, np.int64), 10)
    assert est.numel() == 0


def test_largest_walker_count():
    """2^32 - 1 walkers for one entry (the largest count: ordinals are 32-bit), 4.2e6
    chunk partials merged by a full wave: the sampled walkers at both ends of the
    ordinal range against the oracle, the estimate against the exact value within 5
    standard errors, and 2^32 walkers rejected."""
    a = MATS["cycle31"]
    g, o = _pair(a, 0.5, 21, fp32=True)
    v = np.random.default_rng(8).uniform(0.5, 1.5, a.n)
    m = 2**32 - 1
    est, se = g.entries(v, [3], m)
    st = g.stats()
    assert st["walkers"] == m and st["events"] == st["jumps"] + m
    exact = refs.expm_multiply_v(a.to_scipy(), 0.5, v)[3]
    assert abs(est.item() - exact) < 5 * se.item() and se.item() < 1e-4 * exact
    vv = _v_for(v, True)
    for w0 in (0, m - 500):
        xg, eg, jg, fg = g.trace(v, 3, w0, 500)
        xo, eo, jo, fo, _ = o.trace(vv, 3, w0, 500)
        assert np.array_equal(xg, xo) and np.array_equal(eg, eo) and np.array_equal(jg, jo)
        assert _close(fg, fo, RTOL32)
    with pytest.raises(mc.MCError) as ei:
        g.entries(v, [3], 2**32)
    assert ei.value.code == 1


def test_diagonal_matrix_exact_on_gpu():
    d = np.array([-1.0, 0.0, 0.3, 2.0])
    a = wl.from_dense(np.diag(d))
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 0.7, 1)
    v = np.array([1.0, 2.0, -3.0, 0.5])
    est, se = g.full(v, 100)
    assert np.allclose(est.cpu().numpy(), np.exp(d * 0.7) * v, rtol=1e-15, atol=0)


def test_out_of_range_entry_is_reported():
    a = MATS["sym48"]
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 3)
    v = np.ones(a.n)
    with pytest.raises(mc.MCError) as ei:
        g.entries(v, [1, 48, -1], 10)
    assert ei.value.code == 4
    est, _ = g.entries(v, [1, 2], 10)       # the latched error was cleared
    assert torch.isfinite(est).all()


def test_walk_limit_is_reported():
    a = wl.cycle_graph(8, 50.0)
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 10.0, 1, max_events=64)
    with pytest.raises(mc.MCError) as ei:
        g.entries(np.ones(8), [0], 4)
    assert ei.value.code == 8


def test_fp32_start_value_overflow_taken_by_no_walker():
    """A hub with r t = 100 and d = r: its no-jump value e^{td} v overflows FP32, but no
    walker stays (probability e^{-100}), so the estimate is finite and matches the
    FP64 oracle; the entry must not become 0 * inf = NaN."""
    n = 201
    a = np.zeros((n, n))
    a[0, 1:] = 1.0
    a[1:, 0] = 1.0
    c = wl.from_dense(a)
    v = np.random.default_rng(1).uniform(0.5, 1.5, n)
    g, o = _pair(c, 0.5, 3, fp32=True)
    est, se = g.entries(v, [0, 1, 0], 1000)
    assert np.all(np.isfinite(est.cpu().numpy())) and np.all(np.isfinite(se.cpu().numpy()))
    eo, so = o.estimate(_v_for(v, True), [0, 1, 0], 1000)
    assert _close(est.cpu().numpy(), eo, RTOL32)
    full, _ = g.full(v, 64)
    assert np.all(np.isfinite(full.cpu().numpy()))


def test_fp32_start_value_overflow_taken_by_walkers_is_reported():
    """d t = 90 at a node that walkers seldom leave (r t = 0.01): its stayers' value
    e^{td} v overflows FP32 and the run reports MC_ERR_OVERFLOW."""
    a = np.array([[900.0, 0.1], [0.1, -1.0]])
    c = wl.from_dense(a)
    g = mc.MCExpmv(c.rowptr, c.col, c.val, 0.1, 1, fp32=True)
    with pytest.raises(mc.MCError) as ei:
        g.entries(np.ones(2), [0], 100)
    assert ei.value.code == 9
    h = mc.MCExpmv(c.rowptr, c.col, c.val, 0.1, 1)          # FP64 weights: in range
    est, _ = h.entries(np.ones(2), [0], 100)
    assert np.isfinite(est.item())


@pytest.mark.parametrize("fp32", [False, True])
def test_walker_value_overflow_is_reported_in_every_statistics_tier(fp32):
    """Walkers that jump from node 0 (d = 0) into node 1 (d = 201, or 2001 with FP64
    weights) and hold there pick up e^{d (t - s)} beyond the weight type's range: a
    listed walker's value is infinite, which each per-entry reduction (one lane for
    up to 32 listed walkers, a row of 16 lanes up to 256, the wave beyond) reports
    as MC_ERR_OVERFLOW; the start value K = v[0] stays finite."""
    big = 200.0 if fp32 else 2000.0
    a = np.array([[-1.0, 1.0], [1.0, big]])
    c = wl.from_dense(a)
    for nwalk in (40, 300, 3000):            # about 25, 190 and 1900 listed walkers
        g = mc.MCExpmv(c.rowptr, c.col, c.val, 1.0, 7, fp32=fp32)
        with pytest.raises(mc.MCError) as ei:
            g.entries(np.ones(2), [0], nwalk)
        assert ei.value.code == 9, nwalk
    # a hold short enough to stay in range: no error
    g = mc.MCExpmv(c.rowptr, c.col, c.val, 0.01, 7, fp32=fp32)
    est, _ = g.entries(np.ones(2), [0], 3000)
    assert np.isfinite(est.item())


@pytest.mark.parametrize("kind,code", [("negative", 2), ("nan", 3), ("col", 1), ("rowptr", 1)])
def test_create_rejects_invalid_matrices(kind, code):
    a = np.array([[-1.0, 0.5, 0.0], [0.5, -1.0, 0.5], [0.0, 0.5, -1.0]])
    csr = wl.from_dense(a)
    rowptr, col, val = csr.rowptr.copy(), csr.col.copy(), csr.val.copy()
    if kind == "negative":
        val[1] = -0.5
    elif kind == "nan":
        val[2] = np.nan
    elif kind == "col":
        col[3] = 7
    elif kind == "rowptr":
        rowptr[1] = 5
        rowptr[2] = 2
    with pytest.raises(mc.MCError) as ei:
        mc.MCExpmv(rowptr, col, val, 1.0, 1)
    assert ei.value.code == code
    with pytest.raises(orc.OracleError) as eo:
        Oracle(rowptr, col, val, 1.0, 1)
    assert eo.value.code == code


def test_stream_ordering_on_a_side_stream():
    a = MATS["grid2d_16"]
    v = np.random.default_rng(8).random(a.n)
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 4)
    ref, _ = g.full(v, 500)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        vt = torch.as_tensor(v, device="cuda")
        g.set_stream(s.cuda_stream)
        est = torch.empty(a.n, dtype=torch.float64, device="cuda")
        g.full(vt, 500, est=est, sync=False)
        out = est * 1.0                    # consumer on the same stream
    s.synchronize()
    g.sync()
    assert torch.equal(out, ref)


def test_stream_switch_orders_after_queued_work():
    """Work queued on one stream, then the handle switched to another with no host wait:
    the second run (same chunk-partial scratch) waits for the first, and both results
    equal those of synchronous runs."""
    a = MATS["grid2d_16"]
    v = np.random.default_rng(9).random(a.n)
    idx1 = np.arange(0, a.n, 3, dtype=np.int64)
    idx2 = np.arange(1, a.n, 5, dtype=np.int64)
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 6)
    r1, s1 = [x.clone() for x in g.entries(v, idx1, 70_000)]
    r2, s2 = [x.clone() for x in g.entries(v, idx2, 50_000)]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    vt = torch.as_tensor(v, device="cuda")
    torch.cuda.synchronize()
    g.set_stream(sa.cuda_stream)
    e1 = torch.empty(len(idx1), dtype=torch.float64, device="cuda")
    q1 = torch.empty_like(e1)
    g.entries(vt, idx1, 70_000, est=e1, stderr=q1, sync=False)
    g.set_stream(sb.cuda_stream)
    e2 = torch.empty(len(idx2), dtype=torch.float64, device="cuda")
    q2 = torch.empty_like(e2)
    g.entries(vt, idx2, 50_000, est=e2, stderr=q2, sync=False)
    g.sync()
    sa.synchronize()
    assert torch.equal(e1, r1) and torch.equal(q1, s1)
    assert torch.equal(e2, r2) and torch.equal(q2, s2)


# ------------------------------------------------------ tilted proposal
def test_proposal_tables_and_paths_match_oracle():
    a = MATS["nonsym48"]
    bias = np.random.default_rng(4).normal(0, 0.6, a.nnz).astype(np.float32)
    g, o = _pair(a, 1.0, 55)
    g.set_proposal(bias)
    o.set_proposal(bias)
    tg, to = g.tables(proposal=True), o.tables(proposal=True)
    for key in ("deg", "begin", "col"):
        assert np.array_equal(tg[key], to[key]), key
    for key in ("r", "d", "inv_r"):
        assert np.allclose(tg[key], to[key], rtol=4e-16, atol=0), key
    # thresholds come from a*exp(b): a 1-ulp exp difference may move one by a unit
    assert np.abs(tg["thr"].astype(np.int64) - to["thr"].astype(np.int64)).max() <= 1
    v = np.random.default_rng(5).uniform(0.3, 1.0, a.n)
    for start in (0, 17, 47):
        xg, eg, jg, fg = g.trace(v, start, 0, 4000, proposal=True)
        xo, eo, jo, fo, _ = o.trace(v, start, 0, 4000, proposal=True)
        assert np.array_equal(xg, xo) and np.array_equal(eg, eo) and np.array_equal(jg, jo)
        assert _close(fg, fo, 1e-12)
    est, _ = g.full(v, 2000)
    eo, _ = o.estimate(v, None, 2000, proposal=True)
    assert _close(est.cpu().numpy(), eo, 1e-12)


def test_zero_bias_is_bit_identical_to_plain():
    a = MATS["special40"]
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.2, 8)
    v = np.random.default_rng(1).random(a.n)
    e0, s0 = g.full(v, 1000)
    g.set_proposal(np.zeros(a.nnz, np.float32))
    e1, s1 = g.full(v, 1000)
    assert torch.equal(e0, e1) and torch.equal(s0, s1)
    g.set_proposal(None)
    e2, _ = g.full(v, 1000)
    assert torch.equal(e0, e2)


def test_ground_state_proposal_zero_variance_on_gpu():
    m = 12
    csr = wl.grid2d(m)
    phi, lam = refs.grid2d_ground_state(m)
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    bias = (np.log(phi[csr.col]) - np.log(phi[rows])).astype(np.float32)
    t = 0.6
    g = mc.MCExpmv(csr.rowptr, csr.col, csr.val, t, 8)
    g.set_proposal(bias)
    est, se = g.full(phi, 256)
    est = est.cpu().numpy()
    assert np.allclose(est, np.exp(lam * t) * phi, rtol=2e-6)
    assert np.all(se.cpu().numpy() <= 2e-6 * est)


# ------------------------------------------------- benchmark-size configs
def test_grid2d_config_full_size_parity():
    """32x32 Dirichlet grid, t = 0.1, 16 entries x 1e5 walkers, FP64 (every walker)."""
    w = wl.config_grid2d_entries()
    g, o = _pair(w.a, w.t, 12759)
    est, se = g.entries(w.v, w.idx, w.nwalk)
    eo, so = o.estimate(w.v, w.idx, w.nwalk, threads=8)
    assert _close(est.cpu().numpy(), eo, RTOL64)
    assert np.allclose(se.cpu().numpy(), so, rtol=1e-8)
    ref = refs.grid2d_expm_v(32, w.t, w.v)[w.idx]
    z = (est.cpu().numpy() - ref) / se.cpu().numpy()
    assert np.abs(z).max() < 4.5


def test_grid2d_entries_at_1e3_production_parity():
    """The entries/s measurement's production launch: walker counts from a 1e4-walker
    pilot (1.2 (sigma / (1e-3 x))^2 per entry, up to a few million), all 16 entries in one
    mc_expmv_entries_multi launch; every entry against the oracle with its own count."""
    w = wl.config_grid2d_entries()
    g, o = _pair(w.a, w.t, 12759)
    est0, se0 = g.entries(w.v, w.idx, 10_000)
    x = est0.cpu().numpy()
    sig = se0.cpu().numpy() * np.sqrt(10_000)
    need = np.ceil(1.2 * (sig / (1e-3 * np.abs(x))) ** 2).astype(np.int64)
    assert need.max() > 1_000_000
    est, se = g.entries_multi(w.v, w.idx, need)
    est, se = est.cpu().numpy(), se.cpu().numpy()
    for j, (i, m) in enumerate(zip(w.idx, need)):
        eo, so = o.estimate(w.v, [int(i)], int(m), threads=8)
        assert _close(est[j:j + 1], eo, RTOL64), (j, int(m))
        assert np.allclose(se[j], so, rtol=1e-8), (j, int(m))
    assert np.max(se / np.abs(est)) < 1.2e-3


def test_ba_config_full_size_sampled_parity():
    """BA n=1e5, m=3, full vector with 1e3 walkers/node in FP32 weights: the whole
    vector on the GPU, sampled nodes (hubs included) recomputed by the oracle."""
    w = wl.config_ba_full()
    g = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, fp32=True)
    est, se = g.full(w.v, w.nwalk)
    est = est.cpu().numpy()
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759)
    deg = np.diff(w.a.rowptr)
    hubs = np.argsort(-deg)[:20]
    rand = np.random.default_rng(0).choice(w.a.n, 180, replace=False)
    sample = np.unique(np.concatenate([hubs, rand]))
    eo, _ = o.estimate(_v_for(w.v, True), sample, w.nwalk, threads=8)
    assert _close(est[sample], eo, RTOL32)
    st = g.stats()
    assert st["walkers"] == w.a.n * w.nwalk
    assert st["events"] == st["walkers"] + st["jumps"]


def test_grid3d_config_full_size_sampled_parity():
    """3-D variable-coefficient diffusion, 256^3 (16.7M rows, 1.17e8 entries), t = 0.05,
    full vector with 256 walkers/node in FP32 weights; sampled nodes by the oracle."""
    w = wl.config_grid3d_full()
    g = mc.MCExpmv(w.a.rowptr, w.a.col, w.a.val, w.t, 12759, fp32=True)
    est, se = g.full(w.v, w.nwalk)
    st = g.stats()
    assert st["walkers"] == w.a.n * w.nwalk and st["events"] == st["walkers"] + st["jumps"]
    est = est.cpu().numpy()
    assert np.isfinite(est).all()
    rng = np.random.default_rng(0)
    m = 256
    corner = [0, m - 1, m * m - 1, w.a.n - 1]
    centre = [(m // 2) + m * ((m // 2) + m * (m // 2))]
    sample = np.unique(np.concatenate([corner, centre, rng.choice(w.a.n, 300, replace=False)]))
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759)
    eo, _ = o.estimate(_v_for(w.v, True), sample, w.nwalk, threads=8)
    assert _close(est[sample], eo, RTOL32)


# ------------------------------------------------------------ relabel / LDS
@pytest.mark.parametrize("fp32", [False, True])
def test_relabel_and_hot_rows_do_not_change_results(fp32):
    """Rows stored hot-first (descending exit rate) and the hottest rows staged in LDS:
    paths use original ids in the RNG counter and slot order is kept, so every result
    is bitwise identical to the plain layout."""
    w = wl.config_ba_full(n=20_000)
    a = w.a
    v = np.random.default_rng(3).uniform(0.5, 1.5, a.n)
    base = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32)
    e0, s0 = base.full(v, 300)
    idx = np.array([0, 1, 5, 17, a.n - 1, 4000], np.int64)
    ee0, _ = base.entries(v, idx, 3000)
    t0 = base.trace(v, 3, 0, 2000)
    for relabel, lds in ((1, 0), (1, 4096), (1, 32768)):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32, relabel=relabel,
                       lds_budget=lds)
        e1, s1 = g.full(v, 300)
        assert torch.equal(e0, e1) and torch.equal(s0, s1), (relabel, lds)
        ee1, _ = g.entries(v, idx, 3000)
        assert torch.equal(ee0, ee1)
        t1 = g.trace(v, 3, 0, 2000)
        for x, y in zip(t0, t1):
            assert np.array_equal(x, y)
        tg, tb = g.tables(), base.tables()
        for key in ("r", "d", "inv_r", "deg", "begin", "col", "thr", "alias"):
            assert np.array_equal(tg[key], tb[key]), key


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("lds,block", [(4096, 64), (32768, 64), (32768, 256), (65536, 256)])
def test_hot_rows_in_lds_match_oracle(fp32, lds, block):
    """The kernel that reads the hottest rows from LDS (staged once per block; with
    256-thread blocks the grid holds only blocks that stay resident, each looping
    over many tasks), against the oracle directly: per-walker final state, events
    and jumps identical, per-walker values and the full vector within tolerance,
    on a graph whose hubs sit in the staged rows and whose walks are long enough
    to come back to them."""
    w = wl.config_ba_full(n=20_000)
    a = w.a
    v = np.random.default_rng(5).uniform(0.5, 1.5, a.n)
    t = 3.0
    g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 77, fp32=fp32, relabel=1, lds_budget=lds,
                   walkers_per_block=block)
    o = Oracle(a.rowptr, a.col, a.val, t, 77)
    vo = _v_for(v, fp32)
    tol = RTOL32 if fp32 else RTOL64
    deg = np.diff(a.rowptr)
    hubs = np.argsort(-deg)[:3]
    for start in list(hubs) + [a.n - 1]:
        xg, evg, jug, fg = g.trace(v, int(start), 0, 3000)
        xo, evo, juo, fo, _ = o.trace(vo, int(start), 0, 3000)
        assert np.array_equal(xg, xo) and np.array_equal(evg, evo) and np.array_equal(jug, juo)
        assert _close(fg, fo, tol)
    est, se = g.full(v, 40)
    eo, so = o.estimate(vo, None, 40, threads=8)
    assert _close(est.cpu().numpy(), eo, tol)
    idx = np.concatenate([hubs, [0, 17, a.n - 1]]).astype(np.int64)
    ee, _ = g.entries(v, idx, 5000)
    eeo, _ = o.estimate(vo, idx, 5000, threads=8)
    assert _close(ee.cpu().numpy(), eeo, tol)


def test_relabel_with_proposal_matches_plain_layout():
    a = MATS["nonsym48"]
    bias = np.random.default_rng(4).normal(0, 0.6, a.nnz).astype(np.float32)
    v = np.random.default_rng(5).uniform(0.3, 1.0, a.n)
    g0 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 55)
    g1 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 55, relabel=1, lds_budget=256)
    g0.set_proposal(bias)
    g1.set_proposal(bias)
    e0, _ = g0.full(v, 2000)
    e1, _ = g1.full(v, 2000)
    assert torch.equal(e0, e1)


# ------------------------------------------------------- 64-byte slots
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("mode", [mc.EXACT, mc.STRANG, mc.LIE])
def test_slot_rows_are_bitwise_invisible(fp32, mode):
    """Slots that carry their destinations' rows and d (slot_rows=1) give every path,
    estimate and standard error bit for bit as the separate tables do, and the paths
    match the oracle's."""
    for name in ("special40", "nonsym48", "grid2d_16"):
        a = MATS[name]
        v = np.random.default_rng(6).uniform(-0.5, 1.5, a.n)
        g0 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.1, 17, mode=mode, fp32=fp32, slot_rows=-1)
        g1 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.1, 17, mode=mode, fp32=fp32, slot_rows=1)
        e0, s0 = g0.full(v, 700)
        e1, s1 = g1.full(v, 700)
        assert torch.equal(e0, e1) and torch.equal(s0, s1), name
        idx = np.array([0, 3, a.n - 1, 3], np.int64)
        counts = np.array([5, 3000, 70_000, 1], np.int64)
        m0 = g0.entries_multi(v, idx, counts)
        m1 = g1.entries_multi(v, idx, counts)
        assert torch.equal(m0[0], m1[0]) and torch.equal(m0[1], m1[1]), name
        t0 = g0.trace(v, 3, 0, 1500)
        t1 = g1.trace(v, 3, 0, 1500)
        for x, y in zip(t0, t1):
            assert np.array_equal(x, y), name
    o = Oracle(a.rowptr, a.col, a.val, 1.1, 17, mode=mode, dt=0.03125)
    xo, eo, jo, fo, _ = o.trace(_v_for(v, fp32), 3, 0, 1500)
    assert np.array_equal(t1[0], xo) and np.array_equal(t1[1], eo) and np.array_equal(t1[2], jo)
    assert _close(t1[3], fo, RTOL32 if fp32 else RTOL64)


@pytest.mark.parametrize("fp32", [False, True])
def test_slot_rows_with_relabel_hot_rows_resort_cond_and_proposal(fp32):
    """64-byte slots built from relabelled tables (hot rows in LDS, wave re-sort), with
    first-jump conditioning and with a tilted proposal: bitwise the plain layout."""
    w = wl.config_ba_full(n=20_000)
    a = w.a
    v = np.random.default_rng(3).uniform(0.5, 1.5, a.n)
    idx = np.array([0, 1, 5, 17, a.n - 1, 4000], np.int64)
    bias = np.random.default_rng(4).normal(0, 0.4, a.nnz).astype(np.float32)
    base = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32, slot_rows=-1)
    ref = [base.full(v, 300), base.entries(v, idx, 3000)]
    cbase = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32, cond=True, slot_rows=-1)
    cref = cbase.full(v, 300)
    base.set_proposal(bias)
    pref = base.full(v, 300)
    for kw in (dict(), dict(relabel=1, lds_budget=32768), dict(relabel=1, resort_period=2)):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32, slot_rows=1, **kw)
        for (ea, sa), (eb, sb) in zip(ref, [g.full(v, 300), g.entries(v, idx, 3000)]):
            assert torch.equal(ea, eb) and torch.equal(sa, sb), kw
        gc = mc.MCExpmv(a.rowptr, a.col, a.val, 2.0, 31, fp32=fp32, cond=True, slot_rows=1, **kw)
        ec, sc = gc.full(v, 300)
        assert torch.equal(cref[0], ec) and torch.equal(cref[1], sc), kw
        g.set_proposal(bias)
        ep, sp = g.full(v, 300)
        assert torch.equal(pref[0], ep) and torch.equal(pref[1], sp), kw


def test_slot_rows_automatic_on_large_tables():
    """ER n = 1e6 (tables of 152 MB, above the 64 MiB threshold, so the default picks
    64-byte slots): entries and a trace bitwise equal to the separate tables."""
    a = wl.er_graph(1_000_000, 8.0, 5)
    lam = wl.lambda_max(a)
    a = wl.scaled(a, 1.0 / lam)
    v = np.random.default_rng(2).random(a.n)
    idx = np.random.default_rng(3).choice(a.n, 64).astype(np.int64)
    g0 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 9, slot_rows=-1)
    g1 = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 9)
    e0, s0 = g0.entries(v, idx, 5000)
    e1, s1 = g1.entries(v, idx, 5000)
    assert torch.equal(e0, e1) and torch.equal(s0, s1)
    for x, y in zip(g0.trace(v, int(idx[0]), 0, 3000), g1.trace(v, int(idx[0]), 0, 3000)):
        assert np.array_equal(x, y)


def test_slot_rows_rejects_bad_value():
    a = MATS["sym48"]
    with pytest.raises(mc.MCError):
        mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 1, slot_rows=2)


def test_lds_budget_requires_relabel():
    a = MATS["sym48"]
    with pytest.raises(mc.MCError):
        mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 1, lds_budget=1024)


@pytest.mark.parametrize("fp32", [False, True])
def test_entries_multi_equals_per_count_runs(fp32):
    """One launch with a walker count per entry gives, entry by entry, bitwise what a
    run with that count gives (single chunk, several chunks, ragged tails)."""
    a = MATS["special40"]
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 0.9, 77, fp32=fp32)
    v = np.random.default_rng(3).uniform(-1.0, 2.0, a.n)
    idx = np.array([0, 5, 7, 11, 39, 3, 5, 7], np.int64)
    # 1.5e6 walkers: 2930 (FP64) or 1465 (FP32) chunk partials, merged across waves
    counts = np.array([1, 37, 512, 1025, 5000, 70_000, 2, 1_500_000], np.int64)
    est, se = g.entries_multi(v, idx, counts)
    for j, (i, m) in enumerate(zip(idx, counts)):
        e1, s1 = g.entries(v, [int(i)], int(m))
        assert est[j].item() == e1.item() and se[j].item() == s1.item(), (j, int(m))
    o = Oracle(a.rowptr, a.col, a.val, 0.9, 77)
    eo, so = o.estimate(_v_for(v, fp32), idx[:4], 1025)
    e4, _ = g.entries_multi(v, idx[:4], np.full(4, 1025))
    assert _close(e4.cpu().numpy(), eo, RTOL32 if fp32 else RTOL64)


# ------------------------------------------------------- statistics tiers
@pytest.mark.parametrize("fp32", [False, True])
def test_statistics_tiers_match_oracle(fp32):
    """An entry's listed walkers are summed by one lane (at most 32), one row of 16 lanes
    (at most 256) or the whole wave.  A two-state chain whose start node jumps before t
    with probability 0.55, run with 40 .. 80 and 440 .. 530 walkers, puts chunks (of 512
    walkers with FP64 weights, 1024 with FP32) on both sides of both limits, as counted
    from the oracle's walkers: every estimate and standard error against the oracle."""
    r = -np.log(0.45)
    a = wl.from_dense(np.array([[-r, r], [0.4, -0.4]]))
    t = 1.0
    g, o = _pair(a, t, 123, fp32=fp32)
    v = _v_for(np.array([0.8, 1.7]), fp32)
    counts = np.array(list(range(40, 81, 3)) + list(range(440, 531, 6)), np.int64)
    # listed walkers per chunk, from the oracle's walkers: a walker is listed when its
    # first draw lets it leave (jumps > 0; the band [e0, e^{-rt}) of width 2^-16 e^{-rt}
    # where a listed walker would still stay holds none of these walkers)
    chunk = 1024 if fp32 else 512
    ju = o.trace(v, 0, 0, int(counts.max()))[2]
    js = [int((ju[c:min(c + chunk, m)] > 0).sum()) for m in counts for c in range(0, m, chunk)]
    js = np.array(js)
    assert ((js > 16) & (js <= 32)).any() and ((js > 32) & (js <= 256)).any() and (js > 256).any()
    assert ((js >= 29) & (js <= 32)).any() and ((js >= 33) & (js <= 36)).any(), js
    assert ((js >= 250) & (js <= 256)).any() and ((js >= 257) & (js <= 262)).any(), js
    est, se = g.entries_multi(v, np.zeros(len(counts), np.int64), counts)
    est, se = est.cpu().numpy(), se.cpu().numpy()
    for j, m in enumerate(counts):
        eo, so = o.estimate(v, [0], int(m))
        assert _close(est[j:j + 1], eo, RTOL32 if fp32 else RTOL64), int(m)
        assert np.allclose(se[j], so, rtol=1e-5 if fp32 else 1e-8), int(m)
    # the same counts one at a time (a session of one entry): bitwise the same
    for j in (0, len(counts) - 1):
        e1, s1 = g.entries(v, [0], int(counts[j]))
        assert e1.item() == est[j] and s1.item() == se[j]


# ------------------------------------------------------------ task packing
def _runs(g, v, idx):
    # 512 and 1024 fill a whole LDS list (FP64 / FP32): one entry per session
    out = [g.full(v, m) for m in (1, 37, 300, 512, 1000, 1024, 1500)]
    out += [g.entries(v, idx, 37), g.entries(v, idx, 700)]
    return [(e.clone(), s.clone()) for e, s in out]


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("cond", [False, True])
def test_task_packing_is_bitwise_invisible(fp32, cond):
    """Entries packed into one task (run in several LDS passes when their jumping
    walkers overflow the list) give bitwise what one entry per task gives: per entry
    the walkers, their value slots and the summation tree are the same."""
    for name, t in (("grid2d_16", 2.0), ("special40", 0.9), ("nonsym48", 0.3)):
        a = MATS[name]
        v = np.random.default_rng(6).uniform(-0.5, 2.0, a.n)
        idx = np.concatenate([np.arange(a.n), np.arange(a.n)[::-1], [3, 3, 3]]).astype(np.int64)
        ref = None
        for tw in (1, 0, 2048, 65536):
            g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 8, fp32=fp32, cond=cond, task_walkers=tw)
            res = _runs(g, v, idx)
            if ref is None:
                ref = res
                continue
            for k, ((e0, s0), (e1, s1)) in enumerate(zip(ref, res)):
                assert torch.equal(e0, e1) and torch.equal(s0, s1), (name, tw, k)


def test_task_packing_with_proposal_and_relabel():
    a = MATS["nonsym48"]
    bias = np.random.default_rng(4).normal(0, 0.6, a.nnz).astype(np.float32)
    v = np.random.default_rng(5).uniform(0.3, 1.0, a.n)
    outs = []
    for tw, rl in ((1, 0), (65536, 0), (65536, 1)):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 55, relabel=rl, lds_budget=256 * rl,
                       task_walkers=tw)
        g.set_proposal(bias)
        outs.append([r for m in (50, 900) for r in g.full(v, m)])
    for other in outs[1:]:
        assert all(torch.equal(x, y) for x, y in zip(outs[0], other))


@pytest.mark.parametrize("mode", [mc.EXACT, mc.LIE])
def test_task_packing_matches_oracle(mode):
    """64 entries per task, several passes per task: estimates against the oracle."""
    a = MATS["grid2d_16"]
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.5, 4, mode=mode, dt=0.1, task_walkers=65536)
    o = Oracle(a.rowptr, a.col, a.val, 1.5, 4, mode=mode, dt=0.1)
    v = np.random.default_rng(9).uniform(0.1, 1.0, a.n)
    for m in (37, 600):
        est, se = g.full(v, m)
        eo, so = o.estimate(v, None, m)
        assert _close(est.cpu().numpy(), eo, RTOL64)
        assert _close(se.cpu().numpy(), so, 1e-8)


# ------------------------------------------------------------ wave re-sort
@pytest.mark.parametrize("fp32", [False, True])
def test_wave_resort_does_not_change_results(fp32):
    """Walkers re-sorted by current (relabelled) node every few events, with and
    without LDS hot rows: every path and every estimate bitwise as in input order."""
    w = wl.config_ba_full(n=20_000)
    a = w.a
    v = np.random.default_rng(3).uniform(0.5, 1.5, a.n)
    t = 4.0                                  # long walks: several re-sorts per walker
    base = mc.MCExpmv(a.rowptr, a.col, a.val, t, 31, fp32=fp32)
    e0, s0 = base.full(v, 300)
    idx = np.array([0, 1, 5, 17, a.n - 1, 4000], np.int64)
    ee0, es0 = base.entries(v, idx, 3000)
    t0 = base.trace(v, 3, 0, 2000)
    for period, lds in ((1, 0), (3, 4096), (16, 0)):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 31, fp32=fp32, relabel=1, lds_budget=lds,
                       resort_period=period)
        e1, s1 = g.full(v, 300)
        assert torch.equal(e0, e1) and torch.equal(s0, s1), (period, lds)
        ee1, es1 = g.entries(v, idx, 3000)
        assert torch.equal(ee0, ee1) and torch.equal(es0, es1)
        t1 = g.trace(v, 3, 0, 2000)
        for x, y in zip(t0, t1):
            assert np.array_equal(x, y)


def test_walk_fp32_exp_within_two_ulp():
    """The FP32 weights' own e^x (x log2 e split in two, the hardware exp2, scaling
    by 2^k) against the correctly rounded FP32 value (long double, rounded), within 2
    ulp of FP32 over the normal range, and its ends: 0 below -104 and for -inf,
    denormals near the bottom of the range, +inf above it."""
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(-87.0, 88.7, 200_000), rng.uniform(-1, 1, 50_000),
                        rng.normal(0, 1e-3, 20_000), [0.0, -0.0, 1.0, -1.0, 88.0, -87.0]])
    x = x.astype(np.float32).astype(np.float64)
    y = mc.math_eval("exp_f32", x).cpu().numpy()
    ref = np.exp(x.astype(np.longdouble)).astype(np.float32).astype(np.float64)
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    err = np.abs(y - ref) / ulp
    k = int(np.argmax(err))
    print(f"exp_f32: max error {float(err[k]):.3f} ulp at x = {x[k]!r}", flush=True)
    assert float(err.max()) <= 2.0
    ends = np.array([-np.inf, -104.5, -200.0, 89.0, 100.0, -95.0, -100.0])
    ye = mc.math_eval("exp_f32", ends).cpu().numpy()
    assert ye[0] == 0.0 and ye[1] == 0.0 and ye[2] == 0.0
    assert np.isposinf(ye[3]) and np.isposinf(ye[4])
    for xe, v in zip(ends[5:], ye[5:]):           # FP32 denormals, to their spacing
        r = float(np.float32(np.exp(np.longdouble(xe))))
        assert 0.0 < v and abs(v - r) <= 2 * 2.0 ** -149, (xe, v, r)


@pytest.mark.parametrize("mode,cond,prop", [(mc.LIE, False, False), (mc.EXACT, True, False),
                                            (mc.EXACT, False, True)])
def test_wave_resort_other_walks(mode, cond, prop):
    a = MATS["nonsym48"]
    v = np.random.default_rng(5).uniform(0.3, 1.0, a.n)
    bias = np.random.default_rng(4).normal(0, 0.6, a.nnz).astype(np.float32)
    outs = []
    for rs in (0, 1, 2):
        g = mc.MCExpmv(a.rowptr, a.col, a.val, 2.5, 55, mode=mode, dt=0.1, cond=cond,
                       relabel=1, resort_period=rs)
        if prop:
            g.set_proposal(bias)
        outs.append([r for m in (50, 1500) for r in g.full(v, m)])
    o = Oracle(a.rowptr, a.col, a.val, 2.5, 55, mode=mode, dt=0.1, cond=cond)
    if prop:
        o.set_proposal(bias)
    eo, so = o.estimate(v, None, 50, proposal=prop)
    assert _close(outs[0][0].cpu().numpy(), eo, RTOL64)
    for other in outs[1:]:
        assert all(torch.equal(x, y) for x, y in zip(outs[0], other))


def test_resort_requires_relabel():
    a = MATS["sym48"]
    with pytest.raises(mc.MCError):
        mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 1, resort_period=4)


@pytest.mark.parametrize("fn", ["log", "exp", "one_minus_exp_neg"])
def test_walk_math_within_two_ulp(fn):
    """The walk's own FP64 logarithm (holding times), exponential (FP64 weights) and
    1 - e^{-x} (conditioning) against long-double references, within 3 ulp for the
    logarithm (which loses up to about half an ulp more where e ln2 and the atanh
    series partly cancel) and 2 ulp for the others, on
    seeded arguments across their ranges: every table interval of the logarithm
    (and the 2^-53 grid of U), the exponential's whole range and its limits."""
    rng = np.random.default_rng(11)
    if fn == "log":
        m = rng.integers(0, 2 ** 53, 200_000, dtype=np.uint64)
        u = ((m + np.uint64(1)).astype(np.float64)) * 2.0 ** -53       # the walk's U
        near1 = 1.0 - rng.integers(1, 2 ** 20, 20_000) * 2.0 ** -53
        grid = np.concatenate([1.0 + np.arange(128) / 128.0, 0.75 + np.arange(64) / 256.0])
        edges = np.concatenate([grid, np.nextafter(grid, 0), np.nextafter(grid, 2)]) / 2.0
        x = np.concatenate([u, near1, edges, [1.0, 2.0 ** -53, 0.5, 0.75, 2.0 ** -1022]])
        x = x[(x > 0) & (x <= 1)]
        ref = np.log(x.astype(np.longdouble))
    elif fn == "exp":
        x = np.concatenate([rng.uniform(-700, 700, 100_000), rng.uniform(-1, 1, 50_000),
                            rng.normal(0, 1e-3, 20_000), [0.0, -0.0, 1.0, -1.0, 709.0, -708.0]])
        ref = np.exp(x.astype(np.longdouble))
    else:
        x = np.concatenate([rng.uniform(0, 40, 100_000), 10.0 ** rng.uniform(-12, 0, 50_000),
                            [0.0, 0.34657359027997264, np.nextafter(0.34657359027997264, 0)]])
        ref = -np.expm1(-x.astype(np.longdouble))
    y = mc.math_eval(fn, x).cpu().numpy()
    ulp = np.spacing(np.abs(ref).astype(np.float64))
    ulp = np.where(ref == 0, np.finfo(np.float64).tiny, ulp)
    err = np.abs(y.astype(np.longdouble) - ref) / ulp
    k = int(np.argmax(err))
    print(f"{fn}: max error {float(err[k]):.3f} ulp at x = {x[k]!r}", flush=True)
    assert float(err.max()) <= (3.0 if fn == "log" else 2.0)
