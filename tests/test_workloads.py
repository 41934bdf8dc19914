"""CPU checks of the synthetic input generators against brute-force definitions."""
import numpy as np

from paper_1904_12759_amd import workloads as wl


def test_grid3d_matches_brute_force():
    m = 5
    a = wl.grid3d(m, 1)
    rng = np.random.default_rng(1)
    kap = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=(m, m, m)))
    n = m ** 3
    ref = np.zeros((n, n))
    for z in range(m):
        for y in range(m):
            for x in range(m):
                i = x + m * (y + m * z)
                d = 0.0
                for dz, dy, dx in [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0)]:
                    zz, yy, xx = z + dz, y + dy, x + dx
                    if 0 <= zz < m and 0 <= yy < m and 0 <= xx < m:
                        k2 = kap[zz, yy, xx]
                        f = 2 * kap[z, y, x] * k2 / (kap[z, y, x] + k2)
                        ref[i, xx + m * (yy + m * zz)] = f
                        d -= f
                    else:
                        d -= kap[z, y, x]
                ref[i, i] = d
    assert np.allclose(a.to_dense(), ref, rtol=1e-14, atol=0)
    assert np.array_equal(np.diff(a.rowptr), (ref != 0).sum(1))
    for i in range(n):                                        # columns sorted in each row
        assert np.all(np.diff(a.col[a.rowptr[i]:a.rowptr[i + 1]]) > 0)


def test_grid2d_and_graphs():
    a = wl.grid2d(4)
    d = a.to_dense()
    assert np.allclose(np.diag(d), -4) and np.allclose(d, d.T)
    assert (d[~np.eye(16, dtype=bool)] >= 0).all()
    c = wl.cycle_graph(6, 0.5).to_dense()
    assert np.allclose(c.sum(1), 1.0) and np.allclose(c, c.T)
    e = wl.er_graph(2000, 8.0, 3)
    deg = np.diff(e.rowptr)
    assert 7.0 < deg.mean() < 9.0
    pl = wl.chung_lu_graph(5000, 8.0, 2.5, 3)
    assert pl.to_scipy().max() == 1.0 and np.diff(pl.rowptr).max() > 50


def test_small_world_shape():
    a = wl.small_world(10_000, 0.2, 1)
    dense_check = a.to_scipy()
    assert (dense_check != dense_check.T).nnz == 0          # symmetric
    assert dense_check.diagonal().sum() == 0                 # no loops
    deg = np.diff(a.rowptr)
    assert deg.min() >= 2 and 2.3 < deg.mean() < 2.5
