"""GPU parity of the forward estimator (Lemma 2, Theorem 2, Algorithm 2) against the
CPU oracle, through the C ABI.

Per walker the start node, end node, holding intervals and jumps must be identical and
the value Y within 1e-12 relative (FP64 weights; 1e-5 with FP32 weights).  Per-node
estimates come from FP64 atomics on the GPU (any order) and from compensated sums in
walker order in the oracle, so they agree to 1e-12 relative; standard errors to 1e-8.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle
import paper_1904_12759_amd as mc
from paper_1904_12759_amd import workloads as wl
import refs

pytestmark = pytest.mark.gpu


def _sym(n=40, seed=11):
    return wl.from_dense(refs.random_metzler(n, 0.2, seed, symmetric=True, off_scale=1.0,
                                             diag_scale=1.5))


def _v(n, seed=12):
    return np.random.default_rng(seed).uniform(-1, 2, n)


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) if a.size else 0.0


@pytest.mark.parametrize("mode,fp32", [(mc.EXACT, False), (mc.STRANG, False), (mc.LIE, False),
                                       (mc.EXACT, True), (mc.LIE, True)])
def test_forward_walkers_match_oracle(mode, fp32):
    a = _sym()
    v = _v(a.n)
    vv = np.asarray(v, np.float32).astype(np.float64) if fp32 else v
    t = 0.9
    g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 21, mode=mode, dt=0.2, fp32=fp32)
    o = Oracle(a.rowptr, a.col, a.val, t, 21, mode=mode, dt=0.2)
    # 3000 walkers from ordinal 700: several chunks, a ragged tail, a non-zero base
    gs, ge, gev, gju, gy = g.forward_trace(v, 700, 3000)
    _, _, _, _, (os_, oe, oev, oju, oy) = o.forward(vv, 3700, walkers=True)
    sl = slice(700, 3700)
    np.testing.assert_array_equal(gs, os_[sl])
    np.testing.assert_array_equal(ge, oe[sl])
    np.testing.assert_array_equal(gev, oev[sl])
    np.testing.assert_array_equal(gju, oju[sl])
    assert _rel(gy, oy[sl]) <= (1e-5 if fp32 else 1e-12)


@pytest.mark.parametrize("m", [1, 511, 20_000])
def test_forward_estimates_match_oracle(m):
    a = _sym(64, 13)
    v = _v(a.n, 14)
    t = 0.7
    g = mc.MCExpmv(a.rowptr, a.col, a.val, t, 5)
    o = Oracle(a.rowptr, a.col, a.val, t, 5)
    est, se, tot = g.forward(v, m)
    oest, ose, otot, otse = o.forward(v, m)
    est, se, tot = est.cpu().numpy(), se.cpu().numpy(), tot.cpu().numpy()
    assert np.array_equal(est == 0, oest == 0)
    assert _rel(est, oest) <= 1e-12
    assert _rel(se, ose) <= 1e-8
    assert _rel(tot[0], otot) <= 1e-12
    assert _rel(tot[1], otse) <= 1e-8 or (m == 1 and tot[1] == 0.0)


def test_forward_full_size_sampled():
    """BA n=1e5 m=3 (the backward benchmark's graph), 1e6 forward walkers in the
    configuration the benchmark times: sampled walkers against the oracle one by one,
    and the totals against sum_i x_i within the statistical error."""
    w = wl.config_ba_full()
    a = w.a
    v = np.random.default_rng(2).random(a.n)
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 12759)
    o = Oracle(a.rowptr, a.col, a.val, 1.0, 12759)
    m = 1_000_000
    est, se, tot = g.forward(v, m)
    for w0 in (0, 499_712, m - 300):
        gs, ge, gev, gju, gy = g.forward_trace(v, w0, 300)
        _, _, _, _, (os_, oe, oev, oju, oy) = o.forward(v, w0 + 300, walkers=True)
        sl = slice(w0, w0 + 300)
        np.testing.assert_array_equal(gs, os_[sl])
        np.testing.assert_array_equal(ge, oe[sl])
        np.testing.assert_array_equal(gev, oev[sl])
        assert _rel(gy, oy[sl]) <= 1e-12
    ref = refs.expm_multiply_v(a.to_scipy(), 1.0, v)
    tot = tot.cpu().numpy()
    assert abs(tot[0] - ref.sum()) < 5 * tot[1]
    assert abs(est.sum().item() - tot[0]) < 1e-9 * abs(tot[0])


def test_forward_total_is_reproducible_and_relabel_invariant():
    a = _sym(50, 17)
    v = _v(a.n, 18)
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.1, 9)
    r = mc.MCExpmv(a.rowptr, a.col, a.val, 1.1, 9, relabel=1)
    e1, s1, t1 = g.forward(v, 30_000)
    e1, t1 = e1.clone(), t1.clone()
    e2, s2, t2 = g.forward(v, 30_000)
    e3, s3, t3 = r.forward(v, 30_000)
    _, _, t4 = g.forward(v, 30_000, total_only=True)
    assert torch.equal(t1, t2) and torch.equal(t1, t3) and torch.equal(t1, t4)
    assert _rel(e2.cpu().numpy(), e1.cpu().numpy()) <= 1e-13
    assert _rel(e3.cpu().numpy(), e1.cpu().numpy()) <= 1e-13


def test_forward_cycle_total_is_exact():
    n, beta, t = 33, 0.4, 1.2
    c = wl.cycle_graph(n, beta)
    g = mc.MCExpmv(c.rowptr, c.col, c.val, t, 3)
    est, se, tot = g.forward(np.ones(n), 10_000)
    tot = tot.cpu().numpy()
    exact = n * np.exp(2 * beta * t)
    assert tot[0] == pytest.approx(exact, rel=1e-13) and tot[1] < 1e-10 * exact


def test_forward_rejects_nonsymmetric_and_handles_zero_v():
    a = wl.from_dense(refs.random_metzler(20, 0.3, 4, symmetric=False))
    g = mc.MCExpmv(a.rowptr, a.col, a.val, 1.0, 1)
    with pytest.raises(mc.MCError) as ei:
        g.forward(np.ones(a.n), 100)
    assert ei.value.code == 5
    s = _sym(20, 5)
    h = mc.MCExpmv(s.rowptr, s.col, s.val, 1.0, 1)
    est, se, tot = h.forward(np.zeros(s.n), 1000)
    assert not est.any() and not se.any() and not tot.any()
