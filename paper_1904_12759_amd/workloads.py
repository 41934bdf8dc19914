"""Seeded synthetic inputs: matrices A (CSR), vectors v, entry lists, horizons t.

This module only builds inputs.  It holds none of the estimator's arithmetic
(no rates, weights, tables or walks), so both the HIP library's tests and the
oracle's tests draw their inputs from it.

The workloads stand in for the paper's experiments (Sec. 6), whose graphs
(CONTEST small-world / preferential-attachment generators, SuiteSparse road
and Wikipedia networks) are not available here:

* ``grid2d``  2-D 5-point Dirichlet Laplacian (diag -4, +1 to in-grid neighbours).
* ``ba``      Barabasi-Albert preferential-attachment graph, A = beta * adjacency
              with beta = c / lambda_max (the paper's beta = 1/lambda_max
              normalisation of Sec. 6, scaled by c).
* ``grid3d``  3-D 7-point variable-coefficient diffusion operator (method of
              lines), harmonic-mean face coefficients, Dirichlet boundary.
* ``er`` / ``chung_lu``  Erdos-Renyi and power-law (Chung-Lu) random graphs.
* ``small_world``  Newman-Watts ring with random shortcuts (mean degree 2.4),
              standing in for the paper's small-world networks (Sec. 6, Tables 0, 00).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    rowptr: np.ndarray   # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def n(self) -> int:
        return len(self.rowptr) - 1

    @property
    def nnz(self) -> int:
        return len(self.col)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def from_scipy(m) -> CSR:
    m = m.tocsr()
    m.sort_indices()
    return CSR(np.asarray(m.indptr, np.int64), np.asarray(m.indices, np.int32),
               np.asarray(m.data, np.float64))


def from_dense(a: np.ndarray) -> CSR:
    import scipy.sparse as sp
    return from_scipy(sp.csr_matrix(a))


def _edges_to_adjacency(n: int, u: np.ndarray, w: np.ndarray, scale: float = 1.0) -> CSR:
    """Symmetric 0/1 adjacency (times scale) from undirected edge lists, no loops."""
    import scipy.sparse as sp
    keep = u != w
    u, w = u[keep], w[keep]
    r = np.concatenate([u, w]).astype(np.int64)
    c = np.concatenate([w, u]).astype(np.int64)
    m = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    m.sum_duplicates()
    m.data[:] = scale
    return from_scipy(m)


# ----------------------------------------------------------------- matrices
def grid2d(m: int) -> CSR:
    """2-D 5-point Dirichlet Laplacian on an m x m grid, node = x + m*y."""
    import scipy.sparse as sp
    e = np.ones(m)
    t1 = sp.diags([e[:-1], -2 * e, e[:-1]], [-1, 0, 1])
    eye = sp.identity(m)
    return from_scipy(sp.kron(eye, t1) + sp.kron(t1, eye))


def path_graph(n: int, scale: float = 1.0) -> CSR:
    u = np.arange(n - 1)
    return _edges_to_adjacency(n, u, u + 1, scale)


def cycle_graph(n: int, scale: float = 1.0) -> CSR:
    u = np.arange(n)
    return _edges_to_adjacency(n, u, (u + 1) % n, scale)


def ba_graph(n: int, m: int, seed: int) -> CSR:
    """Barabasi-Albert graph (networkx's generator), unit weights."""
    import networkx as nx
    g = nx.barabasi_albert_graph(int(n), int(m), seed=int(seed))
    import scipy.sparse as sp  # noqa: F401
    a = nx.to_scipy_sparse_array(g, format="csr", dtype=np.float64, nodelist=range(int(n)))
    return from_scipy(a)


def lambda_max(a: CSR) -> float:
    """Largest eigenvalue of a symmetric matrix (Lanczos, FP64)."""
    import scipy.sparse.linalg as sla
    return float(sla.eigsh(a.to_scipy(), k=1, which="LA", tol=1e-10)[0][0])


def scaled(a: CSR, beta: float) -> CSR:
    return CSR(a.rowptr.copy(), a.col.copy(), a.val * beta)


def grid3d(m: int, seed: int, kmin: float = 0.1, kmax: float = 10.0) -> CSR:
    """3-D 7-point variable-coefficient operator on an m^3 grid, node = x + m*(y + m*z).

    Cell coefficients kappa = exp(U[ln kmin, ln kmax]); the coefficient of an
    interior face is the harmonic mean of its two cells, a boundary face uses
    its cell's kappa.  Off-diagonal = face coefficient, diagonal = -sum of the
    six face coefficients (Dirichlet, not scaled by h^2)."""
    rng = np.random.default_rng(seed)
    kap = np.exp(rng.uniform(math.log(kmin), math.log(kmax), size=(m, m, m)))  # [z, y, x]
    n = m ** 3
    # face coefficients along each axis between cell c and c+1: shape m-1 on that axis
    faces = []
    for ax in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        ka, kb = kap[tuple(lo)], kap[tuple(hi)]
        faces.append(2.0 * ka * kb / (ka + kb))
    # per node: the seven entries in column order z-1, y-1, x-1, self, x+1, y+1, z+1
    vals = np.zeros((m, m, m, 7))
    valid = np.zeros((m, m, m, 7), bool)
    diag = np.zeros((m, m, m))
    slot = {(0, -1): 0, (1, -1): 1, (2, -1): 2, (2, 1): 4, (1, 1): 5, (0, 1): 6}
    for ax in range(3):
        f = faces[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        # neighbour at +1 along ax for cells 0..m-2, at -1 for cells 1..m-1
        vals[tuple(lo) + (slot[(ax, 1)],)] = f
        valid[tuple(lo) + (slot[(ax, 1)],)] = True
        vals[tuple(hi) + (slot[(ax, -1)],)] = f
        valid[tuple(hi) + (slot[(ax, -1)],)] = True
        diag[tuple(lo)] -= f
        diag[tuple(hi)] -= f
        # boundary faces use the cell's own coefficient
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = slice(0, 1)
        last[ax] = slice(m - 1, m)
        diag[tuple(first)] -= kap[tuple(first)]
        diag[tuple(last)] -= kap[tuple(last)]
    vals[..., 3] = diag
    valid[..., 3] = True
    vals = vals.reshape(n, 7)
    valid = valid.reshape(n, 7)
    counts = valid.sum(1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    offs = np.array([-m * m, -m, -1, 0, 1, m, m * m], np.int32)
    cols = np.arange(n, dtype=np.int32)[:, None] + offs[None, :]
    return CSR(rowptr, cols[valid], vals[valid])


def small_world(n: int, p: float, seed: int) -> CSR:
    """Newman-Watts small world: a ring (each node joined to its neighbour on either
    side) plus, from every node, a shortcut to a uniform random node with probability
    p; loops and repeated edges dropped.  Mean degree about 2 + 2p (2.4 for p = 0.2)."""
    rng = np.random.default_rng(seed)
    u = np.arange(n, dtype=np.int64)
    ring_w = (u + 1) % n
    has = rng.random(n) < p
    su = u[has]
    sw = rng.integers(0, n, size=len(su))
    return _edges_to_adjacency(n, np.concatenate([u, su]), np.concatenate([ring_w, sw]))


def er_graph(n: int, mean_deg: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, p) with p = mean_deg/(n-1): Binomial edge count, uniform pairs."""
    rng = np.random.default_rng(seed)
    pairs = n * (n - 1) // 2
    p = mean_deg / (n - 1)
    m = rng.binomial(pairs, p)
    u = rng.integers(0, n, size=int(m * 1.02) + 16)
    w = rng.integers(0, n, size=len(u))
    return _edges_to_adjacency(n, u, w)


def chung_lu_graph(n: int, mean_deg: float, gamma: float, seed: int) -> CSR:
    """Power-law random graph: edge endpoints drawn with probability proportional to
    w_i = (i+1)^(-1/(gamma-1)), mean expected degree mean_deg, binarised, no loops."""
    rng = np.random.default_rng(seed)
    w = (np.arange(n) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= mean_deg * n / w.sum()
    p = w / w.sum()
    m = int(round(mean_deg * n / 2))
    u = rng.choice(n, size=m, p=p)
    x = rng.choice(n, size=m, p=p)
    return _edges_to_adjacency(n, u, x)


# ------------------------------------------------------------------ vectors
def uniform_v(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(n)


def bump_v(m: int, seed: int, width: float = 32.0) -> np.ndarray:
    """Gaussian bump at the grid centre plus U[0,1] noise on an m^3 grid."""
    z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    c = (m - 1) / 2.0
    r2 = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    v = np.exp(-r2 / (2.0 * width * width)) + np.random.default_rng(seed).random((m, m, m))
    return v.reshape(-1)


# ------------------------------------------------------------------ configs
@dataclasses.dataclass
class Workload:
    name: str
    a: CSR
    t: float
    v: np.ndarray
    idx: np.ndarray | None      # None: full vector
    nwalk: int                  # walkers per entry / per node
    fp32: bool
    note: str = ""


def config_grid2d_entries(m: int = 32, nwalk: int = 100_000) -> Workload:
    """2-D Dirichlet Laplacian 32x32, t = 0.1, 16 seeded entries x 1e5 walkers, FP64."""
    a = grid2d(m)
    v = uniform_v(a.n, 2)
    idx = np.random.default_rng(3).choice(a.n, 16, replace=False).astype(np.int64)
    return Workload("grid2d_32x32_entries", a, 0.1, v, idx, nwalk, False)


def config_ba_full(n: int = 100_000, m: int = 3, nwalk: int = 1000,
                   c: float = 0.5) -> Workload:
    """BA(n=1e5, m=3, seed 1), A = (0.5/lambda_max) * adjacency, t = 1, v = 1;
    full vector, 1e3 walkers per node, FP32 weights, FP64 reduction."""
    g = ba_graph(n, m, 1)
    lam = lambda_max(g)
    a = scaled(g, c / lam)
    return Workload(f"ba_n{n}_m{m}_full", a, 1.0, np.ones(a.n), None, nwalk, True,
                    note=f"lambda_max={lam:.10g}")


def config_grid3d_full(m: int = 256, nwalk: int = 256) -> Workload:
    """3-D variable-coefficient diffusion 256^3, t = 0.05, bump + noise v, full vector,
    256 walkers per node, FP32."""
    a = grid3d(m, 1)
    return Workload(f"grid3d_{m}_full", a, 0.05, bump_v(m, 2), None, nwalk, True)


def batched_instances(count: int = 64, seed: int = 4, nmin: float = 1e3, nmax: float = 1e6,
                      entries: int = 32, walk_entries: int = 10_000, walk_full: int = 64):
    """Mixed instances: type k mod 4 = ER-entries, ER-full, PL-entries, PL-full;
    n log-uniform in [nmin, nmax], A = adjacency / lambda_max, t ~ U[0.05, 1], v ~ U[0,1]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(10 ** rng.uniform(math.log10(nmin), math.log10(nmax))))
        kind = k % 4
        gseed = 1000 + k
        g = er_graph(n, 8.0, gseed) if kind in (0, 1) else chung_lu_graph(n, 8.0, 2.5, gseed)
        lam = lambda_max(g)
        a = scaled(g, 1.0 / lam)
        t = float(rng.uniform(0.05, 1.0))
        v = np.random.default_rng(2000 + k).random(n)
        if kind in (0, 2):
            idx = np.random.default_rng(3000 + k).choice(n, entries, replace=False)
            out.append(Workload(f"inst{k}", a, t, v, idx.astype(np.int64), walk_entries, False))
        else:
            out.append(Workload(f"inst{k}", a, t, v, None, walk_full, False))
    return out


def stencil7_faces(a: CSR, nx: int, ny: int, nz: int):
    """The face-rate form of a 7-point matrix on an nx x ny x nz grid (node
    i + nx (j + ny k)): fx[x] = a(x, x+1) (0 on the last x-plane), fy[x] = a(x, x+nx),
    fz[x] = a(x, x+nx ny), diag[x] = a(x, x): the entries themselves, copied."""
    n = nx * ny * nz
    assert a.n == n
    rows = np.repeat(np.arange(n), np.diff(a.rowptr))
    col = np.asarray(a.col, np.int64)
    val = np.asarray(a.val, np.float64)
    fx = np.zeros(n)
    fy = np.zeros(n)
    fz = np.zeros(n)
    diag = np.zeros(n)
    d = col - rows
    xs = rows % nx
    ys = (rows // nx) % ny
    m = d == 1
    m &= xs[:] < nx - 1
    fx[rows[m]] = val[m]
    m = (d == nx) & (ys < ny - 1)
    fy[rows[m]] = val[m]
    m = d == nx * ny
    fz[rows[m]] = val[m]
    m = d == 0
    np.add.at(diag, rows[m], val[m])
    return fx, fy, fz, diag
