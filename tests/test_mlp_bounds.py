"""CPU checks of the error bounds the proposal-network GPU tests use (mlp_bounds).

An FP32 emulation of the kernels' arithmetic (bf16 weights, bf16 a1 and dS/dz2
operands, FP32 products and sums in an order of its own, the normalisation by
the FP32 sum of p_e last) must lie inside the bounds element by element, both
against the oracle with the same roundings and against the exact network.  The
same emulation with a plausible slip (a rounding in the wrong place, the
normalised instead of the un-normalised derivative rounded, a transposed W2 in
the backward product, a dropped ReLU mask) must leave the rounded bounds
somewhere: the bounds are tight enough to see such mistakes.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1904_12759_amd import workloads as wl
import mlp_bounds
import refs

f32 = np.float32


def _bf(x):
    return omlp.bf16(x).astype(f32)


def _problem(seed=0, n=120):
    a = wl.from_dense(refs.random_metzler(n, 0.08, seed, False))
    v = np.random.default_rng(seed).uniform(0.2, 1.0, n)
    f = omlp.features(a.rowptr, a.col, a.val, v).astype(f32).astype(np.float64)
    pos, src, dst, pw = omlp.edges(a.rowptr, a.col, a.val)
    rng = np.random.default_rng(seed + 1)
    p = np.concatenate([rng.normal(0, 0.6, 512), rng.normal(0, 0.2, 64),
                        rng.normal(0, 0.15, 4096), rng.normal(0, 0.2, 64),
                        rng.normal(0, 0.3, 64), [0.1]]).astype(f32).astype(np.float64)
    lh = rng.normal(0, 1, n).astype(f32)
    tgt = lh[dst].astype(np.float64) - lh[src].astype(np.float64)
    return f, src, dst, pw, p, lh, len(a.col)


def _emulate(p, feats, src, dst, pw, lh, slip=None):
    """FP32 forward, backward and reduction in the kernels' operand precisions."""
    w1, b1, w2, b2, w3, b3 = (np.asarray(t, f32) for t in omlp.unpack(_bf(p)))
    b3 = f32(b3)
    x = np.concatenate([feats[src], feats[dst]], 1).astype(f32)
    z1 = np.broadcast_to(b1, (len(src), 64)).copy()
    for c in range(8):                                   # sequential FP32, as one lane does
        z1 = (z1 + (x[:, c:c + 1] * w1[:, c][None, :]).astype(f32)).astype(f32)
    a1 = np.maximum(z1, f32(0))
    a1q = _bf(a1)
    z2 = (a1q @ w2.T).astype(f32) + b2
    a2 = np.maximum(z2, f32(0))
    if slip == "round_a2":
        a2 = _bf(a2)
    y = (a2 @ w3).astype(f32) + b3
    th = np.tanh(y * f32(0.125)).astype(f32)
    b = (f32(8) * th).astype(f32)
    tgt = (lh[dst] - lh[src]).astype(f32)
    pe = pw.astype(f32)
    diff = (b - tgt).astype(f32)
    gy = ((f32(2) * pe * diff).astype(f32) * (f32(1) - th * th)).astype(f32)
    dz = np.where(z2 > 0, (gy[:, None] * w3[None, :]).astype(f32), f32(0))
    if slip == "no_mask2":
        dz = (gy[:, None] * w3[None, :]).astype(f32)
    ps32 = pe.sum(dtype=f32)
    dzq = _bf(dz / ps32) * ps32 if slip == "round_normalised" else _bf(dz)
    w2b = w2.T if slip == "transpose_w2" else w2
    gz1 = np.where(z1 > 0, (dzq @ w2b).astype(f32), f32(0))
    S = [gz1.T @ x, gz1.sum(0, dtype=f32), dzq.T @ a1q, dz.sum(0, dtype=f32), a2.T @ gy,
         np.array([gy.sum(dtype=f32)])]
    s = np.concatenate([np.ravel(v).astype(np.float64) for v in S])
    ps = float(ps32)
    lsum = float((pe * diff * diff).astype(f32).sum(dtype=f32))
    return b.astype(np.float64), (s / ps).astype(f32).astype(np.float64), lsum / ps


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("rounded", [True, False])
def test_fp32_emulation_within_bounds(seed, rounded):
    f, src, dst, pw, p, lh, npos = _problem(seed)
    tgt = lh[dst].astype(np.float64) - lh[src].astype(np.float64)
    b, g, loss = _emulate(p, f, src, dst, pw, lh)
    bo, eb, _ = mlp_bounds.forward_bounds(p, f, src, dst, rounded)
    assert np.all(np.abs(b - bo) <= eb)
    lo, go, el, eg = mlp_bounds.gradient_bounds(p, f, src, dst, pw, tgt, npos, rounded)
    assert abs(loss - lo) <= el
    ratio = np.abs(g - go) / eg
    assert np.all(ratio <= 1.0), (int(np.argmax(ratio)), ratio.max())
    if rounded:
        # element-wise: most bounds sit far below one bf16 step of the largest element
        assert np.median(eg) < 0.02 * 2.0 ** -8 * np.abs(go).max()


@pytest.mark.parametrize("slip", ["round_a2", "round_normalised", "transpose_w2", "no_mask2"])
def test_slips_leave_rounded_bounds(slip):
    f, src, dst, pw, p, lh, npos = _problem(2)
    tgt = lh[dst].astype(np.float64) - lh[src].astype(np.float64)
    b, g, _ = _emulate(p, f, src, dst, pw, lh, slip=slip)
    bo, eb, _ = mlp_bounds.forward_bounds(p, f, src, dst, True)
    _, go, _, eg = mlp_bounds.gradient_bounds(p, f, src, dst, pw, tgt, npos, True)
    outside = np.sum(np.abs(g - go) > eg) + np.sum(np.abs(b - bo) > eb)
    assert outside > 0, slip
