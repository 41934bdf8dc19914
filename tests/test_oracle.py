"""Pins of the CPU oracle to what the paper and the mathematics fix.

None of these compare the oracle with itself: the expected values come from
published known-answer vectors, an independent RNG library, dense matrix
exponentials and split products (scipy), spectral closed forms, exact laws of
the jump process (Poisson jump counts, two-state transition probabilities) and
invariants (generator rows, diagonal matrices, t = 0).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import EXACT, LIE, STRANG, Oracle, OracleError
from paper_1904_12759_amd import workloads as wl
import refs

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox
def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert oracle.philox4x32_10(ctr, key).tolist() == expect


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    """rocRAND's host-callable Philox4x32-10 engine is an independent implementation."""
    exe = tmp_path / "rp"
    subprocess.check_call(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "helpers", "rocrand_philox.cpp"), "-o", str(exe)],
                          cwd=str(tmp_path))
    rng = np.random.default_rng(7)
    ctrs = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    ctrs[:, 1] %= 2**30       # rocRAND's offset argument is 4*(c0 | c1 << 32) in 64 bits
    text = "\n".join(" ".join(str(int(x)) for x in row) for row in ctrs) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    got = np.array([[int(x) for x in ln.split()] for ln in out.stdout.strip().splitlines()])
    for row, g in zip(ctrs, got):
        assert oracle.philox4x32_10(row[:4], row[4:]).tolist() == g.tolist()


# ------------------------------------------------------------- alias tables
def _law_from_tables(tb, i):
    """Exact jump law encoded by row i's alias table (thresholds are 2^-32 fixed point)."""
    law = {}
    b, deg = int(tb["begin"][i]), int(tb["deg"][i])
    for s in range(b, b + deg):
        keep = float(tb["thr"][s]) / 2**32
        if tb["alias"][s] == tb["col"][s]:
            keep = 1.0
        law[int(tb["col"][s])] = law.get(int(tb["col"][s]), 0.0) + keep / deg
        law[int(tb["alias"][s])] = law.get(int(tb["alias"][s]), 0.0) + (1 - keep) / deg
    return law


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_alias_reconstructs_jump_law(seed):
    a = refs.random_metzler(40, 0.3, seed, symmetric=False, off_scale=3.0)
    a[5, :] = 0.0                              # a row with no jumps
    a[7, :] = 0.0
    a[7, 3] = 0.25
    a[7, 9] = 0.25                             # a uniform row
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 1)
    tb = o.tables()
    for i in range(a.shape[0]):
        off = a[i].copy()
        off[i] = 0.0
        r = off.sum()
        assert tb["deg"][i] == np.count_nonzero(off > 0)
        assert np.isclose(tb["r"][i], r, rtol=1e-14)
        assert np.isclose(tb["d"][i], a[i, i] + r, rtol=1e-14, atol=1e-15)
        if r == 0:
            continue
        law = _law_from_tables(tb, i)
        for j in range(a.shape[0]):
            assert abs(law.get(j, 0.0) - off[j] / r) <= 2.0**-31, (i, j)


def test_alias_draws_chi2():
    """Empirical jump frequencies of 2e5 walkers that jump exactly once match k_ij."""
    n = 6
    a = np.zeros((n, n))
    a[0, 1:] = [1.0, 2.0, 3.0, 0.5, 7.5]
    csr = wl.from_dense(a)
    t = 50.0  # walker leaves 0 almost surely; states 1..5 have rate 0
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 11)
    x, ev, ju, _, _ = o.trace(np.ones(n), 0, 0, 200_000)
    assert (ju == 1).all()
    counts = np.bincount(x, minlength=n)[1:]
    p = a[0, 1:] / a[0, 1:].sum()
    chi2, pval = stats.chisquare(counts, p * counts.sum())
    assert pval > 1e-4


# ------------------------------------------------------- path-law closed forms
def test_poisson_jump_counts():
    """On a cycle with unit rates both ways the number of jumps in [0,t] is Poisson(2t)."""
    n, t = 17, 1.7
    csr = wl.cycle_graph(n)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 5)
    _, ev, ju, _, _ = o.trace(np.ones(n), 3, 0, 100_000)
    assert (ev == ju + 1).all()
    kmax = 12
    obs = np.bincount(np.minimum(ju, kmax), minlength=kmax + 1)
    pmf = stats.poisson.pmf(np.arange(kmax), 2 * t)
    pmf = np.append(pmf, 1 - pmf.sum())
    chi2, pval = stats.chisquare(obs, pmf * obs.sum())
    assert pval > 1e-4


def test_two_state_terminal_law():
    """Two-state chain 0 -a-> 1, 1 -b-> 0: P(X_t = 0 | X_0 = 0) = (b + a e^{-(a+b)t})/(a+b)."""
    a_, b_, t = 1.3, 0.4, 0.9
    a = np.array([[0.0, a_], [b_, 0.0]])
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 21)
    x, _, _, _, _ = o.trace(np.ones(2), 0, 0, 200_000)
    p00 = (b_ + a_ * np.exp(-(a_ + b_) * t)) / (a_ + b_)
    k = int((x == 0).sum())
    assert stats.binomtest(k, len(x), p00).pvalue > 1e-4


def test_no_jump_probability():
    """P(no jump in [0,t]) = exp(-r t) for the holding-time law Exp(r)."""
    csr = wl.from_dense(np.array([[0.0, 2.5], [0.0, 0.0]]))
    t = 0.3
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 2)
    _, _, ju, _, _ = o.trace(np.ones(2), 0, 0, 100_000)
    k = int((ju == 0).sum())
    assert stats.binomtest(k, len(ju), np.exp(-2.5 * t)).pvalue > 1e-4


def test_walkers_are_independent():
    """The estimator's error model (Sec. 5, sigma / sqrt(M)) needs independent walkers.
    With P(no jump) about 1/2 at the start, the first-event outcomes of neighbouring
    ordinals (2j and 2j+1, 2j+1 and 2j+2) are uncorrelated, for two start nodes and an
    odd first ordinal."""
    csr = wl.from_dense(np.array([[0.0, np.log(2.0)], [0.7, 0.0]]))
    o = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 5)
    for start, w0 in ((0, 0), (0, 1001), (1, 0)):
        _, _, ju, _, _ = o.trace(np.ones(2), start, w0, 40_000)
        j = (ju > 0).astype(float)
        for a, b in ((j[0::2], j[1::2]), (j[1:-1:2], j[2::2])):
            r = np.corrcoef(a, b)[0, 1]
            assert abs(r) < 5.0 / np.sqrt(len(a)), (start, w0, r)


# ----------------------------------------------------------- special cases
def test_diagonal_matrix_is_exact():
    d = np.array([-1.0, 0.0, 0.3, 2.0])
    csr = wl.from_dense(np.diag(d))
    v = np.array([1.0, 2.0, -3.0, 0.5])
    t = 0.7
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 1)
    est, se = o.estimate(v, nwalk=50)
    # every walker returns exp(t a_ii) v_i; the mean of 50 equal values is within an ulp
    assert np.allclose(est, np.exp(d * t) * v, rtol=1e-15, atol=0)
    assert np.all(se <= 1e-15 * np.abs(est))
    x, ev, ju, f, lw = o.trace(v, 3, 0, 10)
    assert np.array_equal(f, np.full(10, np.exp(2.0 * t) * 0.5)) and (ju == 0).all()


def test_generator_preserves_ones():
    """Q with zero row sums: exp(tQ) 1 = 1, and every walker's weight is exactly 1."""
    a = refs.random_metzler(30, 0.4, 3, symmetric=False)
    np.fill_diagonal(a, 0.0)
    for i in range(30):
        s = 0.0
        for j in range(30):
            if j != i and a[i, j] > 0:
                s = s + a[i, j]       # same order as the CSR row
        a[i, i] = -s
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, 2.0, 9)
    est, se = o.estimate(np.ones(30), nwalk=200)
    assert np.array_equal(est, np.ones(30))
    assert np.array_equal(se, np.zeros(30))


@pytest.mark.parametrize("mode", [EXACT, STRANG, LIE])
def test_t_zero_returns_v(mode):
    a = refs.random_metzler(12, 0.5, 4, symmetric=True)
    csr = wl.from_dense(a)
    v = np.random.default_rng(1).random(12)
    o = Oracle(csr.rowptr, csr.col, csr.val, 0.0, 1, mode=mode, dt=0.1)
    est, se = o.estimate(v, nwalk=20)
    assert np.allclose(est, v, rtol=1e-15, atol=0)
    assert np.all(se <= 1e-15 * est)
    _, _, ju, f, _ = o.trace(v, 4, 0, 20)
    assert np.array_equal(f, np.full(20, v[4])) and (ju == 0).all()


# ------------------------------------------------ estimator vs exact values
def _zscores(est, se, ref):
    se = np.where(se > 0, se, 1e-300)
    return (est - ref) / se


@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("seed", [1, 2])
def test_exact_mode_matches_dense_expm(symmetric, seed):
    n = 48
    a = refs.random_metzler(n, 0.15, seed, symmetric=symmetric, off_scale=1.0)
    t = 0.8
    v = np.random.default_rng(seed + 100).uniform(-1, 2, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 1234 + seed)
    est, se = o.estimate(v, nwalk=20_000, threads=4)
    ref = refs.expm_v(a, t, v)
    z = _zscores(est, se, ref)
    assert np.abs(z).max() < 4.5, np.abs(z).max()
    assert abs(np.mean(z ** 2) - 1) < 0.5     # standardized errors have unit variance


@pytest.mark.parametrize("mode,nsteps", [(STRANG, 4), (LIE, 4), (STRANG, 7), (LIE, 3)])
def test_split_modes_match_split_products(mode, nsteps):
    """Theorem 1: the STRANG/LIE estimators are unbiased for the split products."""
    n = 24
    a = refs.random_metzler(n, 0.25, 7, symmetric=True, off_scale=1.5, diag_scale=2.0)
    t = 1.0
    v = np.random.default_rng(8).uniform(0.5, 1.5, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 77, mode=mode, dt=t / nsteps)
    assert o.ngrid == nsteps
    est, se = o.estimate(v, nwalk=40_000, threads=4)
    ref = (refs.strang_v if mode == STRANG else refs.lie_v)(a, t, nsteps, v)
    z = _zscores(est, se, ref)
    assert np.abs(z).max() < 4.5
    # the splitting error is resolvable: the exact exponential is rejected at this M
    exact = refs.expm_v(a, t, v)
    assert np.mean(_zscores(est, se, exact) ** 2) > 5.0


def test_cycle_closed_form():
    n, c, t = 20, 0.7, 1.5
    csr = wl.cycle_graph(n, c)
    v = np.random.default_rng(5).random(n)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 3)
    est, se = o.estimate(v, nwalk=20_000, threads=4)
    ref = refs.cycle_expm_v(n, c, 0.0, t, v)
    assert np.abs(_zscores(est, se, ref)).max() < 4.5


def test_path_closed_form():
    n, c, t = 15, 0.9, 1.0
    csr = wl.path_graph(n, c)
    v = np.random.default_rng(6).random(n)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 4)
    est, se = o.estimate(v, nwalk=20_000, threads=4)
    ref = refs.path_expm_v(n, c, t, v)
    assert np.abs(_zscores(est, se, ref)).max() < 4.5


def test_grid2d_config_closed_form():
    """The 32x32 Dirichlet grid at t = 0.1 against its Kronecker/sine closed form."""
    w = wl.config_grid2d_entries(nwalk=20_000)
    ref = refs.grid2d_expm_v(32, w.t, w.v)
    dense = refs.expm_v(w.a.to_dense(), w.t, w.v)
    assert np.abs(ref - dense).max() < 1e-12
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, w.t, 12759)
    est, se = o.estimate(w.v, w.idx, w.nwalk, threads=4)
    assert np.abs(_zscores(est, se, ref[w.idx])).max() < 4.5


def test_statistical_error_scales_as_inverse_sqrt():
    """Sec. 5: the standard error decays as M^{-1/2} (Fig. 4 slope -1/2)."""
    w = wl.config_grid2d_entries()
    o = Oracle(w.a.rowptr, w.a.col, w.a.val, 1.0, 31)
    ses = []
    for m in (1000, 4000, 16000, 64000):
        _, se = o.estimate(w.v, w.idx[:4], m, threads=4)
        ses.append(se)
    ses = np.array(ses)
    ratios = ses[:-1] / ses[1:]
    assert np.all(np.abs(ratios - 2.0) < 0.25), ratios


# ----------------------------------------------------- determinism / layout
def test_threads_duplicates_and_full_agree():
    a = refs.random_metzler(30, 0.3, 5, symmetric=True)
    csr = wl.from_dense(a)
    v = np.random.default_rng(2).random(30)
    o = Oracle(csr.rowptr, csr.col, csr.val, 0.9, 5)
    idx = np.array([3, 7, 3, 29, 0])
    e1, s1 = o.estimate(v, idx, 500, threads=1)
    e4, s4 = o.estimate(v, idx, 500, threads=3)
    assert np.array_equal(e1, e4) and np.array_equal(s1, s4)
    assert e1[0] == e1[2]
    ef, sf = o.estimate(v, None, 500, threads=2)
    assert np.array_equal(ef[idx], e1) and np.array_equal(sf[idx], s1)


def test_instance_and_seed_change_stream():
    a = refs.random_metzler(10, 0.5, 5, symmetric=True)
    csr = wl.from_dense(a)
    v = np.ones(10)
    base = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 5).trace(v, 2, 0, 100)
    other_inst = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 5, instance=1).trace(v, 2, 0, 100)
    other_seed = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 6).trace(v, 2, 0, 100)
    assert not np.array_equal(base[3], other_inst[3])
    assert not np.array_equal(base[3], other_seed[3])


# ------------------------------------------------------------- validation
def _csr_case(kind):
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
        rowptr[-1] = 99
    return rowptr, col, val


@pytest.mark.parametrize("kind,code", [("negative", 2), ("nan", 3), ("col", 1), ("rowptr", 1)])
def test_rejects_invalid_matrices(kind, code):
    rowptr, col, val = _csr_case(kind)
    with pytest.raises(OracleError) as ei:
        Oracle(rowptr, col, val, 1.0, 1)
    assert ei.value.code == code


def test_rejects_bad_horizon_and_entries():
    rowptr, col, val = _csr_case("ok")
    for t in (-1.0, np.nan, np.inf):
        with pytest.raises(OracleError):
            Oracle(rowptr, col, val, t, 1)
    o = Oracle(rowptr, col, val, 1.0, 1)
    with pytest.raises(OracleError) as ei:
        o.estimate(np.ones(3), np.array([0, 5]), 10)
    assert ei.value.code == 4


def test_walk_limit():
    csr = wl.cycle_graph(8, 50.0)
    o = Oracle(csr.rowptr, csr.col, csr.val, 10.0, 1, max_events=64)
    with pytest.raises(OracleError) as ei:
        o.estimate(np.ones(8), np.array([0]), 4)
    assert ei.value.code == 8


# -------------------------------------------------------- tilted proposal
def test_zero_bias_is_plain():
    a = refs.random_metzler(25, 0.3, 9, symmetric=False)
    csr = wl.from_dense(a)
    v = np.random.default_rng(1).random(25)
    o = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 19)
    o.set_proposal(np.zeros(csr.nnz, np.float32))
    for s in (0, 13):
        p = o.trace(v, s, 0, 300, proposal=False)
        q = o.trace(v, s, 0, 300, proposal=True)
        for x, y in zip(p, q):
            assert np.array_equal(x, y)


def test_ground_state_bias_gives_zero_variance():
    """Doob h-transform with the Dirichlet grid's Perron vector phi: with v = phi and
    b_ij = log phi_j - log phi_i every walker returns exp(lambda t) phi_i."""
    m = 12
    csr = wl.grid2d(m)
    phi, lam = refs.grid2d_ground_state(m)
    rows = np.repeat(np.arange(csr.n), np.diff(csr.rowptr))
    bias = (np.log(phi[csr.col]) - np.log(phi[rows])).astype(np.float32)
    # float32 biases: use the h they actually encode on every edge (exact potential form)
    t = 0.6
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 8)
    o.set_proposal(bias)
    est, se = o.estimate(phi, None, 64, proposal=True)
    # float32 rounding of b breaks the telescoping by <= 1e-7 per jump
    assert np.allclose(est, np.exp(lam * t) * phi, rtol=2e-6)
    assert np.all(se <= 2e-6 * est)
    est0, se0 = o.estimate(phi, None, 64)
    assert np.median(se0 / est0) > 100 * np.median(se / est)


def test_random_bias_is_unbiased():
    n = 30
    a = refs.random_metzler(n, 0.2, 12, symmetric=False)
    csr = wl.from_dense(a)
    v = np.random.default_rng(3).uniform(0.2, 1.0, n)
    bias = np.random.default_rng(4).normal(0.0, 0.7, csr.nnz).astype(np.float32)
    t = 0.7
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 99)
    o.set_proposal(bias)
    est, se = o.estimate(v, None, 20_000, proposal=True, threads=4)
    ref = refs.expm_v(a, t, v)
    assert np.abs(_zscores(est, se, ref)).max() < 4.5


@pytest.mark.parametrize("tilted", [False, True])
def test_exact_second_moment_matches_oracle_samples(tilted):
    """The exact second-moment formula (used to price walker-steps) against the
    oracle's empirical mean of f^2 (var + mean^2) within statistical error."""
    n = 25
    a = refs.random_metzler(n, 0.25, 13, symmetric=False)
    csr = wl.from_dense(a)
    v = np.random.default_rng(1).uniform(0.2, 1.0, n)
    t = 0.6
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 3)
    bias = None
    if tilted:
        bias = np.random.default_rng(2).normal(0, 0.5, csr.nnz).astype(np.float32)
        o.set_proposal(bias)
    m2 = refs.second_moment_exact(csr, t, v, bias)
    nw = 40_000
    for i in (0, 7, 19):
        _, _, _, f, _ = o.trace(v, i, 0, nw, proposal=tilted)
        f2 = f * f
        emp = f2.mean()
        sd = f2.std() / np.sqrt(nw)
        assert abs(emp - m2[i]) < 4.5 * sd, (i, emp, m2[i], sd)


# --------------------------------------------------- forward estimator
# Lemma 2 / Theorem 2 / Algorithm 2: starts drawn with probability |v_j|/V, the
# value V sign(v_j) W credited to the state where the walk ends.
def test_forward_cycle_total_is_exact():
    """On a cycle with weight beta, d = 2 beta everywhere, so every walker carries
    exactly V e^{2 beta t}: the mean of Y is n e^{2 beta t} = (1, e^{tA} 1) with zero
    variance, and the per-node estimates add up to it."""
    n, beta, t = 12, 0.3, 1.3
    c = wl.cycle_graph(n, beta)
    o = Oracle(c.rowptr, c.col, c.val, t, 5)
    est, se, tot, tse = o.forward(np.ones(n), 5000)
    exact = n * np.exp(2 * beta * t)
    assert tot == pytest.approx(exact, rel=1e-14) and tse < 1e-12 * exact
    assert est.sum() == pytest.approx(exact, rel=1e-13)
    ref = refs.cycle_expm_v(n, beta, 0.0, t, np.ones(n))
    assert np.abs((est - ref) / se).max() < 4.5


def test_forward_matches_dense_expm_symmetric():
    n = 40
    a = refs.random_metzler(n, 0.2, 11, symmetric=True, off_scale=1.0)
    t = 0.8
    v = np.random.default_rng(12).uniform(-1, 2, n)       # negative entries carry a sign
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 31)
    est, se, tot, tse = o.forward(v, 400_000)
    ref = refs.expm_v(a, t, v)
    z = _zscores(est, se, ref)
    assert np.abs(z).max() < 4.5 and abs(np.mean(z ** 2) - 1) < 0.5
    assert abs(tot - ref.sum()) < 4.5 * tse


def test_forward_estimates_transpose_action():
    """Without symmetry the forward walks estimate e^{tA^T} v (Kolmogorov forward
    equation); for this matrix e^{tA} v is many standard errors away."""
    n = 30
    a = refs.random_metzler(n, 0.3, 21, symmetric=False, off_scale=1.5)
    t = 1.0
    v = np.random.default_rng(22).uniform(0.2, 1.0, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 32)
    est, se, _, _ = o.forward(v, 400_000)
    zt = _zscores(est, se, refs.expm_v(a.T, t, v))
    assert np.abs(zt).max() < 4.5
    assert np.mean(_zscores(est, se, refs.expm_v(a, t, v)) ** 2) > 25.0


def test_forward_start_law():
    """Starts follow |v_j| / V (chi-square), nodes with v_j = 0 are never drawn, and with
    t = 0 every walker stays at its start, so each Y is exactly V sign(v_start)."""
    n = 16
    a = refs.random_metzler(n, 0.3, 5, symmetric=True)
    csr = wl.from_dense(a)
    v = np.random.default_rng(6).uniform(-1, 1, n)
    v[[3, 9]] = 0.0
    V = np.abs(v).sum()
    m = 200_000
    o = Oracle(csr.rowptr, csr.col, csr.val, 0.0, 7)
    est, se, tot, tse, (st, en, ev, ju, y) = o.forward(v, m, walkers=True)
    assert np.array_equal(st, en) and (ju == 0).all()
    np.testing.assert_allclose(y, V * np.sign(v[st]), rtol=1e-14)
    assert len(np.unique(y)) <= 2
    counts = np.bincount(st, minlength=n)
    assert counts[3] == 0 and counts[9] == 0
    p = np.abs(v) / V
    keep = p > 0
    chi2 = (((counts - m * p) ** 2)[keep] / (m * p[keep])).sum()
    assert chi2 < 45.0        # 13 degrees of freedom: P(chi2 > 45) < 1e-4
    z = _zscores(est, np.where(se > 0, se, 1.0), v)
    assert np.abs(z).max() < 4.5


@pytest.mark.parametrize("mode,nsteps", [(STRANG, 4), (LIE, 4), (LIE, 3)])
def test_forward_split_modes_match_split_products(mode, nsteps):
    """With the grid coefficients read in reverse time order, the forward STRANG/LIE
    estimators are unbiased for the same split products as the backward ones (symmetric A)."""
    n = 24
    a = refs.random_metzler(n, 0.25, 7, symmetric=True, off_scale=1.5, diag_scale=2.0)
    t = 1.0
    v = np.random.default_rng(8).uniform(0.5, 1.5, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 78, mode=mode, dt=t / nsteps)
    est, se, _, _ = o.forward(v, 600_000)
    ref = (refs.strang_v if mode == STRANG else refs.lie_v)(a, t, nsteps, v)
    z = _zscores(est, se, ref)
    assert np.abs(z).max() < 4.5
    assert np.mean(_zscores(est, se, refs.expm_v(a, t, v)) ** 2) > 5.0


def test_forward_zero_vector():
    csr = wl.cycle_graph(6, 1.0)
    o = Oracle(csr.rowptr, csr.col, csr.val, 1.0, 1)
    est, se, tot, tse = o.forward(np.zeros(6), 100)
    assert not est.any() and not se.any() and tot == 0.0 and tse == 0.0


# ------------------------------------------- first-jump conditioning (cond)
# The no-jump event of the start node (probability e^{-rt}) is integrated
# exactly; only walks that jump before t are sampled.
def _rate_and_d(a):
    off = a - np.diag(np.diag(a))
    r = off.sum(1)
    return r, np.diag(a) + r


@pytest.mark.parametrize("symmetric", [True, False])
def test_conditioned_matches_dense_expm(symmetric):
    n = 40
    a = refs.random_metzler(n, 0.15, 41, symmetric=symmetric, off_scale=1.0)
    t = 0.7
    v = np.random.default_rng(42).uniform(-1, 2, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 43, cond=True)
    est, se = o.estimate(v, nwalk=20_000, threads=4)
    ref = refs.expm_v(a, t, v)
    # rows without jumps are deterministic: exact up to rounding
    det = se <= 1e-13 * np.abs(ref)
    np.testing.assert_allclose(est[det], ref[det], rtol=1e-13)
    z = _zscores(est[~det], se[~det], ref[~det])
    assert np.abs(z).max() < 4.5 and abs(np.mean(z ** 2) - 1) < 0.5


@pytest.mark.parametrize("mode,nsteps", [(STRANG, 4), (LIE, 3)])
def test_conditioned_split_modes(mode, nsteps):
    n = 24
    a = refs.random_metzler(n, 0.25, 7, symmetric=True, off_scale=1.5, diag_scale=2.0)
    t = 1.0
    v = np.random.default_rng(8).uniform(0.5, 1.5, n)
    csr = wl.from_dense(a)
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 79, mode=mode, dt=t / nsteps, cond=True)
    est, se = o.estimate(v, nwalk=40_000, threads=4)
    ref = (refs.strang_v if mode == STRANG else refs.lie_v)(a, t, nsteps, v)
    assert np.abs(_zscores(est, se, ref)).max() < 4.5


def test_conditioned_second_moment_is_exact():
    """E[f_c] = x and E[f_c^2] = p0^2 K^2 + 2 p0 K (x - p0 K) + q (m2 - p0 K^2), with
    p0 = e^{-rt}, q = 1 - p0, K = e^{dt} v_i, x = (e^{tA}v)_i and m2 the plain walk's
    exact second moment: the sampled values of the conditioned walker match both."""
    n = 25
    a = refs.random_metzler(n, 0.25, 13, symmetric=False)
    csr = wl.from_dense(a)
    v = np.random.default_rng(1).uniform(0.2, 1.0, n)
    t = 0.6
    o = Oracle(csr.rowptr, csr.col, csr.val, t, 3, cond=True)
    x = refs.expm_v(a, t, v)
    m2 = refs.second_moment_exact(csr, t, v)
    r, d = _rate_and_d(a)
    nw = 40_000
    for i in (0, 7, 19):
        p0 = np.exp(-r[i] * t)
        q = 1 - p0
        k = np.exp(d[i] * t) * v[i]
        m2c = p0 ** 2 * k ** 2 + 2 * p0 * k * (x[i] - p0 * k) + q * (m2[i] - p0 * k ** 2)
        _, _, ju, f, _ = o.trace(v, i, 0, nw)
        assert (ju >= 1).all()                       # every sampled walk jumps
        assert abs(f.mean() - x[i]) < 4.5 * f.std() / np.sqrt(nw)
        f2 = f * f
        assert abs(f2.mean() - m2c) < 4.5 * f2.std() / np.sqrt(nw), (i, f2.mean(), m2c)


def test_conditioned_reduces_variance_on_low_rate_nodes():
    """Where the start node rarely leaves (e^{-rt} near 1) the jump/no-jump choice
    dominates the plain variance; conditioning removes it."""
    g = wl.ba_graph(2000, 3, 5)
    a = wl.scaled(g, 0.5 / wl.lambda_max(g))
    v = np.random.default_rng(6).random(a.n)
    deg = np.diff(a.rowptr)
    idx = np.where(deg == 3)[0][:20]
    plain = Oracle(a.rowptr, a.col, a.val, 1.0, 7)
    cond = Oracle(a.rowptr, a.col, a.val, 1.0, 7, cond=True)
    _, se_p = plain.estimate(v, idx, 20_000, threads=4)
    _, se_c = cond.estimate(v, idx, 20_000, threads=4)
    assert np.median(se_p / se_c) > 2.0


def test_conditioned_diagonal_and_rate_zero_rows():
    a = np.diag([-0.5, 0.3, 1.0])
    csr = wl.from_dense(a)
    v = np.array([1.0, 2.0, -1.0])
    o = Oracle(csr.rowptr, csr.col, csr.val, 1.5, 1, cond=True)
    est, se = o.estimate(v, nwalk=10)
    np.testing.assert_allclose(est, np.exp(1.5 * np.diag(a)) * v, rtol=1e-15)
    assert not se.any()


def test_conditioning_threshold_selects_nodes():
    """With cond_max_rt = theta, start nodes with r t <= theta take the conditioned
    walk and the others the plain one, walker for walker."""
    g = wl.ba_graph(300, 2, 9)
    a = wl.scaled(g, 0.8 / wl.lambda_max(g))
    v = np.random.default_rng(10).random(a.n)
    t = 1.0
    r = np.zeros(a.n)
    np.add.at(r, np.repeat(np.arange(a.n), np.diff(a.rowptr)), a.val)
    theta = float(np.quantile(r * t, 0.7))
    mixed = Oracle(a.rowptr, a.col, a.val, t, 11, cond=True, cond_max_rt=theta)
    allc = Oracle(a.rowptr, a.col, a.val, t, 11, cond=True)
    plain = Oracle(a.rowptr, a.col, a.val, t, 11)
    low = np.where(r * t < 0.99 * theta)[0][:5]
    high = np.where(r * t > 1.01 * theta)[0][:5]
    assert len(low) and len(high)
    for i in low:
        assert np.array_equal(mixed.trace(v, i, 0, 200)[3], allc.trace(v, i, 0, 200)[3])
    for i in high:
        assert np.array_equal(mixed.trace(v, i, 0, 200)[3], plain.trace(v, i, 0, 200)[3])


# ---------------------------------------------------- randomised lattice (first event)
def _lattice_words(key, start, w, bits, inst=0):
    """The first-event words of the randomised rank-1 lattice, from its definition:
    the point j of the Korobov lattice (1, a, a^2 mod B), j = w mod B written in
    `bits` binary digits and read backwards, shifted modulo 1 by the replicate's
    Philox draw (counter 0xFFFFFFFE, w >> bits, start, instance)."""
    B = 1 << bits
    a = 119 if bits == 9 else 149
    g = [1, a, (a * a) % B]
    sh = oracle.philox4x32_10([0xFFFFFFFE, w >> bits, start, inst], key)
    j = int(format(w % B, f"0{bits}b")[::-1], 2)
    frac = [(j * gk % B) / B for gk in g]                  # the lattice point in [0,1)^3
    shift = [((int(sh[0]) << 32) | int(sh[1])) / 2.0 ** 64, int(sh[2]) / 2.0 ** 32,
             int(sh[3]) / 2.0 ** 32]
    return [(f + s) % 1.0 for f, s in zip(frac, shift)]


@pytest.mark.parametrize("bits", [9, 10])
def test_lattice_first_event_stratifies_the_jump_choice(bits):
    """Within a replicate of B walkers the first-event uniforms are the lattice points
    shifted modulo 1, so the number of walkers whose first holding time outlasts t is
    B e^{-rt} rounded down or up, exactly; and every replicate's walkers reach the
    states the plain walk reaches (single-jump paths from the start's neighbours)."""
    a = wl.cycle_graph(9, 0.7)
    t = 0.45
    o = Oracle(a.rowptr, a.col, a.val, t, 21, qmc=True, qmc_bits=bits)
    v = np.arange(1.0, 10.0)
    B = 1 << bits
    r = 1.4                                                 # two neighbours at rate 0.7
    p0 = np.exp(-r * t)
    for start in (0, 4):
        x, ev, ju, f, _ = o.trace(v, start, 0, 3 * B)
        for c in range(3):
            stay = int((ju[c * B:(c + 1) * B] == 0).sum())
            assert stay in (int(np.floor(B * p0)), int(np.ceil(B * p0))), (c, stay, B * p0)


@pytest.mark.parametrize("count", [256, 128, 64])
def test_lattice_prefix_of_a_replicate_is_stratified(count):
    """The first 2^k walkers of a replicate take the 2^k-point sub-lattice (radical-
    inverse order), so a run with fewer walkers per node than a replicate holds is
    still stratified: of `count` walkers, floor or ceil of count e^{-rt} stay."""
    a = wl.cycle_graph(9, 0.7)
    t = 0.45
    o = Oracle(a.rowptr, a.col, a.val, t, 23, qmc=True, qmc_bits=9)
    v = np.arange(1.0, 10.0)
    p0 = np.exp(-1.4 * t)
    for start in (0, 3, 8):
        x, ev, ju, f, _ = o.trace(v, start, 0, count)
        stay = int((ju == 0).sum())
        assert stay in (int(np.floor(count * p0)), int(np.ceil(count * p0))), (start, stay)


def test_lattice_first_event_words_follow_the_definition():
    """The walker's first event, as the oracle takes it, is the shifted lattice point:
    no-jump exactly when -log U / r >= t with U from the first coordinate, and the
    jump target the alias draw of the other two (checked on a star graph whose
    centre jumps to leaf `slot` with the slot word)."""
    n = 6
    dense = np.zeros((n, n))
    dense[0, 1:] = [0.5, 0.5, 0.5, 0.5, 0.5]               # uniform row: slot = leaf
    a = wl.from_dense(dense)
    t = 0.9
    seed = 33
    key = [seed & 0xFFFFFFFF, seed >> 32]
    o = Oracle(a.rowptr, a.col, a.val, t, seed, qmc=True, qmc_bits=9)
    v = np.arange(1.0, 7.0)
    x, ev, ju, f, _ = o.trace(v, 0, 0, 1500)
    for w in range(0, 1500, 7):
        u, us, _ = _lattice_words(key, 0, w, 9)
        m = int(u * 2.0 ** 53)                              # the top 53 bits of the word
        U = (m + 1) * 2.0 ** -53
        holds = -np.log(U) / 2.5 >= t
        assert holds == (ju[w] == 0), w
        if not holds:
            assert x[w] == 1 + int(us * 5), w               # floor(slot word * deg)


@pytest.mark.parametrize("mode,symmetric", [(EXACT, True), (EXACT, False), (STRANG, True)])
def test_lattice_estimate_is_unbiased_and_its_error_calibrated(mode, symmetric):
    """Over independent seeds (independent shifts) the lattice estimates average to
    the dense reference (expm, or the Strang product), and the replicate standard
    error matches the estimates' spread: with R = 8 replicate means the z-scores
    follow Student's t with R - 1 = 7 degrees of freedom, E[z^2] = 7/5."""
    n = 20
    dense = refs.random_metzler(n, 0.25, 51, symmetric=symmetric)
    t = 0.8
    a = wl.from_dense(dense)
    v = np.random.default_rng(52).uniform(0.2, 1.0, n)
    ref = refs.expm_v(dense, t, v) if mode == EXACT else refs.strang_v(dense, t, 4, v)
    zs = []
    for seed in range(40):
        o = Oracle(a.rowptr, a.col, a.val, t, 1000 + seed, mode=mode, dt=t / 4, qmc=True,
                   qmc_bits=9)
        est, se = o.estimate(v, None, 8 * 512, threads=4)
        zs.append((est - ref) / se)
    z = np.array(zs)
    assert abs(z.mean()) < 4.5 * np.sqrt(1.4 / z.size)
    assert abs(np.mean(z * z) - 1.4) < 0.3, np.mean(z * z)


def test_lattice_reduces_variance():
    """On the 32x32 grid at t = 0.1 (most walkers never leave their start node) the
    lattice's spread over seeds is several times below the plain walk's at the same
    walker count."""
    g = wl.grid2d(32)
    v = wl.uniform_v(g.n, 2)
    idx = np.array([0, 100, 500, 1023, 333])
    ests = {False: [], True: []}
    for seed in range(24):
        for q in (False, True):
            o = Oracle(g.rowptr, g.col, g.val, 0.1, 500 + seed, qmc=q, qmc_bits=9)
            ests[q].append(o.estimate(v, idx, 4096, threads=4)[0])
    var_p = np.var(np.array(ests[False]), axis=0)
    var_q = np.var(np.array(ests[True]), axis=0)
    assert np.all(var_q < var_p) and np.median(var_p / var_q) > 4, var_p / var_q


def test_lattice_standard_error_from_replicate_means():
    """The replicate standard error by its definition, from the traced walker values:
    se^2 = R/(R-1) sum_c (n_c/M)^2 (m_c - mean)^2 over the R replicates (the last one
    partial), and the i.i.d. formula when a single replicate holds every walker."""
    a = wl.grid2d(6)
    v = np.random.default_rng(3).random(a.n)
    o = Oracle(a.rowptr, a.col, a.val, 0.6, 8, qmc=True, qmc_bits=9)
    for m in (3 * 512 + 100, 512, 300):
        est, se = o.estimate(v, [7], m)
        f = o.trace(v, 7, 0, m)[3]
        assert abs(est[0] - f.mean()) <= 1e-14 * abs(f.mean())
        if m > 512:
            reps = [f[c:c + 512] for c in range(0, m, 512)]
            r = len(reps)
            acc = sum((len(x) / m) ** 2 * (x.mean() - f.mean()) ** 2 for x in reps)
            want = np.sqrt(acc * r / (r - 1))
        else:
            want = f.std(ddof=1) / np.sqrt(m)
        assert abs(se[0] - want) <= 1e-10 * want, (m, se[0], want)


# ---------------------------------------------------- inverse-CDF jump rule
def test_cdf_jump_rule_follows_its_definition():
    """With the inverse-CDF rule the first jump goes to the first neighbour (CSR order)
    whose running sum of rates exceeds u r, u = o2 / 2^32 from the walker's first Philox
    draw: checked walker by walker on a row with unequal rates."""
    dense = np.zeros((5, 5))
    dense[0, 1:] = [0.3, 1.1, 0.05, 0.8]
    dense[1:, 0] = 0.2
    a = wl.from_dense(dense)
    seed = 77
    key = [seed & 0xFFFFFFFF, seed >> 32]
    t = 5.0
    o = Oracle(a.rowptr, a.col, a.val, t, seed, cdf_jump=True)
    x, ev, ju, f, _ = o.trace(np.ones(5), 0, 0, 400)
    rates = dense[0, 1:]
    r = rates.sum()
    cum = np.cumsum(rates)
    for w in range(400):
        o2 = int(oracle.philox4x32_10([0, w, 0, 0], key)[2])
        k = int(np.searchsorted(cum, (o2 / 2.0 ** 32) * r, side="right"))
        assert ju[w] >= 1
        if ju[w] == 1:
            assert x[w] == 1 + min(k, 3), w


def test_cdf_jump_frequencies_match_the_jump_law():
    dense = np.zeros((6, 6))
    dense[0, 1:] = [0.5, 2.0, 0.25, 1.0, 0.25]
    a = wl.from_dense(dense)
    o = Oracle(a.rowptr, a.col, a.val, 50.0, 3, cdf_jump=True)
    x, ev, ju, f, _ = o.trace(np.ones(6), 0, 0, 40_000)   # every walker jumps once (rows 1-5 absorb)
    counts = np.bincount(x, minlength=6)[1:]
    p = dense[0, 1:] / dense[0, 1:].sum()
    chi2 = stats.chisquare(counts, p * counts.sum())
    assert chi2.pvalue > 1e-4, chi2


@pytest.mark.parametrize("symmetric", [True, False])
def test_cdf_jump_matches_dense_expm(symmetric):
    n = 40
    dense = refs.random_metzler(n, 0.15, 71, symmetric=symmetric, off_scale=1.0)
    a = wl.from_dense(dense)
    t = 0.8
    v = np.random.default_rng(72).uniform(-1, 2, n)
    o = Oracle(a.rowptr, a.col, a.val, t, 73, cdf_jump=True)
    est, se = o.estimate(v, nwalk=20_000, threads=4)
    ref = refs.expm_v(dense, t, v)
    z = _zscores(est, se, ref)
    assert np.abs(z).max() < 4.5 and abs(np.mean(z ** 2) - 1) < 0.5
