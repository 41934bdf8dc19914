"""FP64 reference of the learned-proposal network and its training step.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by the tests to
check the HIP kernels' features, forward pass, gradients and Adam update.

Variance reduction by importance sampling is the remedy the paper names for
the statistical error (Sec. 5).  The proposal tilts the jump rates of edge
i -> j by exp(b_ij) (see oracle.c); the network predicts b_ij from node
features:

  node features  f_i = [log1p(deg_i), r_i, v_i, log1p(mean of deg_j over the
                 jump targets j of i)], each standardised over the nodes
                 (population standard deviation; 1 when it is 0)
  edge input     x = [f_i ; f_j]                                  (8)
  network        a1 = relu(W1 x + b1)                            (64)
                 a2 = relu(W2 a1 + b2)                           (64)
                 y  = w3 . a2 + b3,  b = 8 tanh(y / 8)
  loss           sum_e p_e (b_e - b*_e)^2 / sum_e p_e,  p_e = a_ij / r_i,
                 b*_e = log h_j - log h_i with h = sqrt(m2), m2 the per-node
                 second moment of W v[X_t] measured by plain runs.

Where the bfloat16 roundings sit.  The products run with bfloat16 operands
and FP32 accumulation, so three kinds of value are rounded to bfloat16: the
weights, the hidden activations a1 (the operand of the 64x64 product), and
the back-propagated derivative at z2 (the operand of the two 64x64 products
of the backward pass, dW2 and dL/da1).  The derivative that is rounded is the
per-edge one of the un-normalised sum  sum_e p_e (b_e - b*_e)^2; the division
by sum_e p_e is applied to the summed gradient.  `bf=True` applies exactly
these roundings; `bf=False` is the exact network in FP64.  Parameter vector
layout (4801 floats): W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

H = 64
NIN = 8
NPARAM = H * NIN + H + H * H + H + H + 1
TANH_SCALE = 8.0


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, np.float64)
    o = 0
    w1 = p[o:o + H * NIN].reshape(H, NIN); o += H * NIN
    b1 = p[o:o + H]; o += H
    w2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return w1, b1, w2, b2, w3, b3


def pack(w1, b1, w2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(w1), b1, np.ravel(w2), b2, w3, [b3]])


def edges(rowptr, col, val):
    """CSR positions of the jump edges (positive off-diagonal entries) with their
    source row, target and jump probability a_ij / r_i."""
    rowptr = np.asarray(rowptr)
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    col = np.asarray(col)
    val = np.asarray(val, np.float64)
    m = (col != rows) & (val > 0)
    pos = np.nonzero(m)[0]
    r = np.zeros(n)
    np.add.at(r, rows[pos], val[pos])
    p = val[pos] / r[rows[pos]]
    return pos, rows[pos], col[pos], p


def features(rowptr, col, val, v) -> np.ndarray:
    """Standardised node features, shape (n, 4)."""
    n = len(rowptr) - 1
    pos, src, dst, _ = edges(rowptr, col, val)
    deg = np.bincount(src, minlength=n).astype(np.float64)
    r = np.zeros(n)
    np.add.at(r, src, np.asarray(val, np.float64)[pos])
    nsum = np.zeros(n)
    np.add.at(nsum, src, deg[dst])
    mean_nb = np.divide(nsum, deg, out=np.zeros(n), where=deg > 0)
    raw = np.stack([np.log1p(deg), r, np.asarray(v, np.float64), np.log1p(mean_nb)], axis=1)
    mu = raw.mean(0)
    sd = raw.std(0)
    sd = np.where(sd > 0, sd, 1.0)
    return (raw - mu) / sd


def targets_from_stats(est, se, nwalk, src, dst, tiny=1e-300):
    """b*_e = log h_dst - log h_src, h = sqrt(second moment of the walker value)."""
    est = np.asarray(est, np.float64)
    se = np.asarray(se, np.float64)
    var = se * se * nwalk
    m2 = var * (nwalk - 1) / nwalk + est * est
    lh = 0.5 * np.log(np.maximum(m2, tiny))
    return lh[dst] - lh[src]


def forward(p, feats, src, dst, bf=True):
    w1, b1, w2, b2, w3, b3 = unpack(bf16(p) if bf else p)
    f = np.asarray(feats, np.float64)
    x = np.concatenate([f[src], f[dst]], axis=1)          # (E, 8)
    z1 = x @ w1.T + b1
    a1 = np.maximum(z1, 0.0)
    a1q = bf16(a1) if bf else a1
    z2 = a1q @ w2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ w3 + b3
    th = np.tanh(y / TANH_SCALE)
    b = TANH_SCALE * th
    cache = (x, z1, a1q, z2, a2, th, (w1, b1, w2, b2, w3, b3))
    return b, cache


def loss_and_grad(p, feats, src, dst, pw, tgt, bf=True, cache=False):
    """Weighted squared error and its gradient w.r.t. the parameter vector.

    Back-propagation runs on the un-normalised sum  S = sum_e p_e (b_e - b*_e)^2
    (per-edge derivatives e_*), and loss and gradient are S and dS/dtheta
    divided by sum_e p_e.  With cache=True the intermediate values are returned
    too (a dict), for deriving the kernels' rounding-error bounds."""
    b, (x, z1, a1q, z2, a2, th, (w1, b1, w2, b2, w3, b3)) = forward(p, feats, src, dst, bf)
    pw = np.asarray(pw, np.float64)
    ps = pw.sum()
    tgt = np.asarray(tgt, np.float64)
    diff = b - tgt
    lsum = float((pw * diff * diff).sum())
    e_y = 2.0 * pw * diff * (1.0 - th * th)              # dS/dy per edge
    e_z2 = np.outer(e_y, w3) * (z2 > 0)                  # dS/dz2 per edge
    e_z2q = bf16(e_z2) if bf else e_z2
    e_z1 = (e_z2q @ w2) * (z1 > 0)                       # dS/dz1 per edge
    g = pack(e_z1.T @ x, e_z1.sum(0), e_z2q.T @ a1q, e_z2.sum(0), a2.T @ e_y, e_y.sum()) / ps
    loss = lsum / ps
    if not cache:
        return loss, g
    return loss, g, dict(x=x, z1=z1, a1q=a1q, z2=z2, a2=a2, th=th, b=b, diff=diff, e_y=e_y,
                         e_z2=e_z2, e_z2q=e_z2q, e_z1=e_z1, lsum=lsum, ps=ps,
                         w=(w1, b1, w2, b2, w3, b3))


def adam(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015), bias-corrected; step counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
