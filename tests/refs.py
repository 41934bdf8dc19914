"""Deterministic references the oracle and the GPU path are pinned to.

Everything here is an independent route to the quantity the Monte Carlo
estimator targets: dense matrix exponentials (scipy's scaling-and-squaring
Pade ``expm``), the paper's split products written as dense matrix products
(Eq. (deff) Lie, Eq. (eq_general1) Strang), spectral closed forms for graphs
whose eigenvectors are known (cycle: Fourier; path and Dirichlet grids: sine
transform), and Al-Mohy/Higham ``expm_multiply`` for large sparse cases.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as la


def expm_v(a: np.ndarray, t: float, v: np.ndarray) -> np.ndarray:
    return la.expm(t * a) @ v


def split_parts(a: np.ndarray):
    """A = D - L with L the Laplacian of the off-diagonal part (paper Sec. 2)."""
    off = a - np.diag(np.diag(a))
    lap = np.diag(off.sum(1)) - off
    dvec = np.diag(a) + off.sum(1)
    return dvec, lap


def strang_v(a: np.ndarray, t: float, nsteps: int, v: np.ndarray) -> np.ndarray:
    """(e^{dt D/2} e^{-dt L} e^{dt D/2})^N v, Eq. (eq_general1)."""
    dvec, lap = split_parts(a)
    dt = t / nsteps
    h = np.exp(dt * dvec / 2)
    step = h[:, None] * la.expm(-dt * lap) * h[None, :]
    x = v.copy()
    for _ in range(nsteps):
        x = step @ x
    return x


def lie_v(a: np.ndarray, t: float, nsteps: int, v: np.ndarray) -> np.ndarray:
    """(e^{-dt L} e^{dt D})^N v, Eq. (deff)."""
    dvec, lap = split_parts(a)
    dt = t / nsteps
    step = la.expm(-dt * lap) * np.exp(dt * dvec)[None, :]
    x = v.copy()
    for _ in range(nsteps):
        x = step @ x
    return x


def cycle_expm_v(n: int, c: float, diag: float, t: float, v: np.ndarray) -> np.ndarray:
    """exp(tA) v for A = c*adjacency(cycle) + diag*I via the DFT (A is circulant)."""
    k = np.arange(n)
    lam = diag + 2 * c * np.cos(2 * np.pi * k / n)
    return np.real(np.fft.ifft(np.exp(t * lam) * np.fft.fft(v)))


def path_expm_v(n: int, c: float, t: float, v: np.ndarray) -> np.ndarray:
    """exp(tA) v for A = c*adjacency(path) via its sine eigenbasis."""
    k = np.arange(1, n + 1)
    s = np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(k, k) / (n + 1))
    lam = 2 * c * np.cos(np.pi * k / (n + 1))
    return s @ (np.exp(t * lam) * (s @ v))


def grid2d_expm_v(m: int, t: float, v: np.ndarray) -> np.ndarray:
    """exp(tA) v for the m x m Dirichlet 5-point Laplacian: A = T(+)T with T the
    1-D tridiag(1,-2,1), so exp(tA) = E (x) E with E = S diag(e^{t mu}) S."""
    k = np.arange(1, m + 1)
    s = np.sqrt(2.0 / (m + 1)) * np.sin(np.pi * np.outer(k, k) / (m + 1))
    mu = -2 + 2 * np.cos(np.pi * k / (m + 1))
    e = s @ np.diag(np.exp(t * mu)) @ s
    x = v.reshape(m, m)          # node = x + m*y  ->  row y, column x
    return (e @ x @ e.T).reshape(-1)


def grid2d_ground_state(m: int):
    """Perron vector phi (positive) and eigenvalue of the m x m Dirichlet Laplacian."""
    k = np.arange(1, m + 1)
    s1 = np.sin(np.pi * k / (m + 1))
    phi = np.outer(s1, s1).reshape(-1)
    lam = -4 + 4 * np.cos(np.pi / (m + 1))
    return phi, lam


def expm_multiply_v(a_sparse, t: float, v: np.ndarray) -> np.ndarray:
    import scipy.sparse.linalg as sla
    return sla.expm_multiply(t * a_sparse, v)


def random_metzler(n: int, density: float, seed: int, symmetric: bool,
                   diag_scale: float = 1.0, off_scale: float = 1.0) -> np.ndarray:
    """Dense random matrix with non-negative off-diagonal entries."""
    rng = np.random.default_rng(seed)
    off = rng.random((n, n)) * off_scale
    mask = rng.random((n, n)) < density
    off = off * mask
    np.fill_diagonal(off, 0.0)
    if symmetric:
        off = np.triu(off, 1)
        off = off + off.T
    a = off + np.diag(rng.uniform(-1.0, 1.0, n) * diag_scale)
    return a


def second_moment_exact(a, t: float, v: np.ndarray, bias=None) -> np.ndarray:
    """E[f^2] per start node for the plain (bias None) or tilted walk, exactly.

    Feynman-Kac with jump factors: for rates q_ij, a factor g_ij per jump and a
    potential V, E[exp(int V) prod g  u(X_t)] = exp(t G) u with G_ij = q_ij g_ij,
    G_ii = V_i - sum_j q_ij.  The squared estimator of the tilted walk has
    q = a e^{b}, g = e^{-2b}, V = 2 d~, so G_ij = a_ij e^{-b_ij} and
    G_ii = 2 d~_i - r~_i (d~ = d + r~ - r); b = 0 gives A + diag(d)."""
    import scipy.sparse as sp
    n = a.n
    rows = np.repeat(np.arange(n), np.diff(a.rowptr))
    off = (a.col != rows) & (a.val > 0)
    diag = np.zeros(n)
    np.add.at(diag, rows[a.col == rows], a.val[a.col == rows])
    r = np.zeros(n)
    np.add.at(r, rows[off], a.val[off])
    d = diag + r
    b = np.zeros(a.nnz) if bias is None else np.asarray(bias, np.float32).astype(np.float64)
    at = a.val[off] * np.exp(b[off])
    rt = np.zeros(n)
    np.add.at(rt, rows[off], at)
    dt = d + (rt - r)
    g = sp.csr_matrix((a.val[off] * np.exp(-b[off]), (rows[off], a.col[off])), shape=(n, n))
    g = g + sp.diags(2 * dt - rt)
    return expm_multiply_v(g.tocsr(), t, np.asarray(v, np.float64) ** 2)
