"""Splitting errors of the two products the STRANG and LIE modes are unbiased for
(Theorem 1, Eqs. (eq_general1), (deff)), computed densely on a small-world graph, against
what Sec. 5 derives: both splittings converge with order 2 for the total
communicability (1, e^A 1) because (1, D L 1) - (1, L D 1) = 0, the Lie product only with
order 1 for a single entry, and the Strang error of the total is about |(1, D L D 1)| dt^2.
CPU only; these references also price the MC points of the splitting study in bench.py."""
import numpy as np

from paper_1904_12759_amd import workloads as wl
import refs


def _slope(dts, errs):
    return np.polyfit(np.log(dts), np.log(errs), 1)[0]


def test_splitting_orders_small_world():
    a = wl.small_world(100, 0.2, 3).to_dense()
    n = a.shape[0]
    one = np.ones(n)
    exact = refs.expm_v(a, 1.0, one)
    dts = np.array([1 / 8, 1 / 16, 1 / 32, 1 / 64])
    tc_s, tc_l, x_s, x_l = [], [], [], []
    for dt in dts:
        nsteps = int(round(1 / dt))
        s = refs.strang_v(a, 1.0, nsteps, one)
        l = refs.lie_v(a, 1.0, nsteps, one)
        tc_s.append(abs(s.sum() - exact.sum()))
        tc_l.append(abs(l.sum() - exact.sum()))
        x_s.append(abs(s[0] - exact[0]))
        x_l.append(abs(l[0] - exact[0]))
    assert 1.8 < _slope(dts, tc_s) < 2.2
    assert 1.8 < _slope(dts, tc_l) < 2.2
    assert 1.8 < _slope(dts, x_s) < 2.2
    assert 0.8 < _slope(dts, x_l) < 1.2
    # leading Strang term of the total: within a factor 2 of |(1, D L D 1)| dt^2
    dvec, lap = refs.split_parts(a)
    lead = abs(one @ (dvec * (lap @ (dvec * one)))) * dts ** 2
    ratio = np.array(tc_s) / lead
    assert np.all((ratio > 0.05) & (ratio < 2.0)), ratio
