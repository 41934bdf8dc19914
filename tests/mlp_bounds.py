"""Per-element bounds on how far the proposal network's GPU kernels may lie from
the FP64 oracle (`oracle/mlp.py`), by running error analysis.

Every quantity of the network carries the oracle's value X and a bound E_X on
|X_gpu - X|, propagated through the arithmetic the kernels do:

* FP32 sums of m terms (VALU loops, shuffles, MFMA accumulation, in any order)
  err by at most gamma(m) * sum|terms|, gamma(m) = m u / (1 - m u), u = 2^-24;
  one FP32 product errs by u |product|; bf16 x bf16 products are exact in FP32.
* ReLU is 1-Lipschitz; where |z| <= E_z the mask itself is uncertain, and a
  backward value gated by it may be either 0 or the full value.
* A bf16 rounding of a value known to within E is either the oracle's
  rounding or a neighbour: the bound is the largest change of bf16() over
  [X - E, X + E] (bf16 is monotone), zero when no rounding boundary lies in
  that interval.
* tanhf adds a few FP32 ulps (4 allowed); y/8 and 8 th are exact.

With `rounded=True` the oracle applies the kernels' bf16 roundings (weights,
a1, the per-edge dS/dz2) and the bound holds only FP32 arithmetic and the
rare roundings that can fall on either side of a boundary: an element-wise
check at the scale of each element's own terms.  With `rounded=False` the
oracle is the exact network, and the bound adds each rounding's actual error
|bf16(X) - X| (the quantisation budget), so the kernel is also checked
against the unrounded network.

`npos` is the number of CSR positions the kernel visited: a lane's sequential
chain of FP32 additions is at most that long (plus shuffle and merge levels).
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as omlp

U = 2.0 ** -24
TANH_ULPS = 4.0
TINY = 2.0 ** -126


def gamma(m):
    return m * U / (1.0 - m * U)


def q_err(x, e, rounded):
    """Bound on |bf16(x_gpu) - X_oracle| for |x_gpu - x| <= e."""
    qx = omlp.bf16(x)
    out = np.maximum(np.abs(omlp.bf16(x - e) - qx), np.abs(omlp.bf16(x + e) - qx))
    if not rounded:
        out = out + np.abs(qx - x)
    return out


def mul_err(a, ea, b, eb):
    """|a_gpu b_gpu (rounded) - a b| for |a_gpu - a| <= ea, |b_gpu - b| <= eb."""
    aa, bb = np.abs(a), np.abs(b)
    return aa * eb + bb * ea + ea * eb + U * (aa + ea) * (bb + eb)


def relu_err(z, ez):
    """Forward: 1-Lipschitz, exactly 0 where z is certainly negative."""
    return np.where(z < -ez, 0.0, ez)


def gated_err(z, ez, val, eval_):
    """A backward value gated by the mask z > 0: where the mask is certain the
    value's own error, where not the whole value may appear or vanish."""
    sure = np.abs(z) > ez
    on = z > 0
    return np.where(sure, np.where(on, eval_, 0.0), np.abs(val) + eval_)


def weight_errs(p, rounded):
    """Bounds on the GPU's bf16 weights against the oracle's weights."""
    p = np.asarray(p, np.float64)
    e = np.zeros_like(p) if rounded else np.abs(omlp.bf16(p) - p)
    return omlp.unpack(e)


def forward_bounds(p, feats, src, dst, rounded):
    """(b_oracle, E_b, intermediates) for the inference kernel."""
    b, (x, z1, a1q, z2, a2, th, (w1, b1, w2, b2, w3, b3)) = omlp.forward(p, feats, src, dst,
                                                                        bf=rounded)
    ew1, eb1, ew2, eb2, ew3, eb3 = weight_errs(p, rounded)
    ax = np.abs(x)
    # layer 1: z = b1 + sum_c w1 x (8 products, 9 additions in FP32)
    ez1 = ax @ ew1.T + eb1 + gamma(omlp.NIN + 1) * (np.abs(b1) + eb1 + ax @ (np.abs(w1) + ew1).T)
    a1 = np.maximum(z1, 0.0)
    ea1 = relu_err(z1, ez1)
    ea1q = q_err(a1, ea1, rounded)
    # layer 2: MFMA over 64 bf16 products (exact) with FP32 accumulation, + b2
    aa1 = np.abs(a1q)
    ez2 = (ea1q @ np.abs(w2).T + aa1 @ ew2.T + ea1q @ ew2.T + eb2
           + gamma(omlp.H + 1) * ((aa1 + ea1q) @ (np.abs(w2) + ew2).T + np.abs(b2) + eb2))
    ea2 = relu_err(z2, ez2)
    # layer 3: y = b3 + sum w3 a2 (FP32 products and sums)
    aa2 = np.abs(a2)
    ey = (ea2 @ np.abs(w3) + aa2 @ ew3 + ea2 @ ew3 + eb3
          + gamma(omlp.H + 2) * ((aa2 + ea2) @ (np.abs(w3) + ew3) + abs(b3) + eb3))
    eth = ey / omlp.TANH_SCALE + TANH_ULPS * U * np.abs(th) + TINY
    eb = omlp.TANH_SCALE * eth
    return b, eb, dict(x=x, z1=z1, ez1=ez1, a1q=a1q, ea1q=ea1q, z2=z2, ez2=ez2, a2=a2, ea2=ea2,
                       th=th, eth=eth, eb=eb)


def gradient_bounds(p, feats, src, dst, pw, tgt, npos, rounded):
    """(loss, grad, E_loss, E_grad) of the training kernel and its reduction:
    per-wave FP32 partials of the un-normalised sums, summed in FP64, divided by
    the summed FP32 p_e, cast to FP32."""
    loss, g, c = omlp.loss_and_grad(p, feats, src, dst, pw, tgt, bf=rounded, cache=True)
    _, _, fb = forward_bounds(p, feats, src, dst, rounded)
    w1, b1, w2, b2, w3, b3 = c["w"]
    ew1, eb1, ew2, eb2, ew3, eb3 = weight_errs(p, rounded)
    pw = np.asarray(pw, np.float64)
    tgt = np.asarray(tgt, np.float64)
    L = npos + 64                       # longest FP32 addition chain of a lane, plus merges
    gL = gamma(L)
    th, eth = c["th"], fb["eth"]
    # per-edge scalars: target (FP32 difference of FP32 log h), p_e (FP32 of a double ratio)
    etgt = U * np.abs(tgt)
    epe = (U + 2.0 ** -50) * pw
    diff = c["diff"]
    ediff = fb["eb"] + etgt + U * (np.abs(diff) + fb["eb"] + etgt)
    th2 = th * th
    eth2 = mul_err(th, eth, th, eth)
    om = 1.0 - th2
    eom = eth2 + U * (np.abs(om) + eth2)
    t2 = 2.0 * pw * diff
    et2 = 2.0 * mul_err(pw, epe, diff, ediff)
    e_y = c["e_y"]
    egy = mul_err(t2, et2, om, eom)
    # dS/dz2 = gy w3 where z2 > 0; its bf16 rounding is the MFMA operand
    prod = np.outer(e_y, w3)
    eprod = mul_err(e_y[:, None], egy[:, None], w3[None, :], ew3[None, :])
    edz = gated_err(c["z2"], fb["ez2"], prod, eprod)
    edzq = q_err(c["e_z2"], edz, rounded)
    dzq = c["e_z2q"]
    # dS/dz1 = W2^T dzq (MFMA, FP32 accumulation) where z1 > 0
    adzq = np.abs(dzq)
    s1 = dzq @ w2
    es1 = (edzq @ np.abs(w2) + adzq @ ew2 + edzq @ ew2
           + gamma(omlp.H) * ((adzq + edzq) @ (np.abs(w2) + ew2)))
    egz1 = gated_err(c["z1"], fb["ez1"], s1, es1)
    gz1 = c["e_z1"]
    x = c["x"]
    ax = np.abs(x)
    a1q, ea1q = c["a1q"], fb["ea1q"]
    a2, ea2 = c["a2"], fb["ea2"]
    aa1 = np.abs(a1q)
    aa2 = np.abs(a2)
    age = np.abs(e_y)
    agz1 = np.abs(gz1)
    e_z2 = c["e_z2"]
    # un-normalised sums over the edges and their bounds
    S = [gz1.T @ x, gz1.sum(0), dzq.T @ a1q, e_z2.sum(0), a2.T @ e_y, np.array([e_y.sum()])]
    A = [agz1.T @ ax, agz1.sum(0), adzq.T @ aa1, np.abs(e_z2).sum(0), aa2.T @ age,
         np.array([age.sum()])]          # sums of |terms|, for the oracle's own FP64 error
    E = [egz1.T @ ax + gamma(L + 1) * ((agz1 + egz1).T @ ax),
         egz1.sum(0) + gL * (agz1 + egz1).sum(0),
         adzq.T @ ea1q + edzq.T @ aa1 + edzq.T @ ea1q + gL * ((adzq + edzq).T @ (aa1 + ea1q)),
         edz.sum(0) + gL * (np.abs(e_z2) + edz).sum(0),
         aa2.T @ egy + ea2.T @ age + ea2.T @ egy + gamma(L + 1) * ((aa2 + ea2).T @ (age + egy)),
         np.array([egy.sum() + gL * (age + egy).sum()])]
    s = np.concatenate([np.ravel(v) for v in S])
    a = np.concatenate([np.ravel(v) for v in A])
    es = np.concatenate([np.ravel(v) for v in E])
    ps = c["ps"]
    eps_ = epe.sum() + gL * pw.sum()
    assert eps_ < 0.5 * ps
    # S_gpu / ps_gpu in FP64, then cast to FP32; plus the oracle's own rounding
    eg = es / (ps - eps_) + np.abs(s) * eps_ / (ps * (ps - eps_))
    eg = eg + U * (np.abs(g) + eg) + 1e-12 * a / ps + 1e-300
    # loss: sum p diff diff in FP32 over the edges, same normalisation
    ldiff = np.abs(diff)
    pd = pw * diff                                        # (p_e diff) diff, two FP32 products
    epd = mul_err(pw, epe, diff, ediff)
    el = mul_err(pd, epd, diff, ediff).sum() + gL * ((pw + epe) * (ldiff + ediff) ** 2).sum()
    lsum = c["lsum"]
    eloss = el / (ps - eps_) + abs(lsum) * eps_ / (ps * (ps - eps_))
    eloss = eloss + U * (abs(loss) + eloss) + 1e-12 * abs(loss)
    return loss, g, eloss, eg
