"""Pins of the FP64 proposal-network oracle (oracle/mlp.py), CPU only."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_1904_12759_amd import workloads as wl
import refs


def _problem(seed=0, n=30):
    a = refs.random_metzler(n, 0.25, seed, symmetric=False)
    csr = wl.from_dense(a)
    v = np.random.default_rng(seed).random(n)
    f = mlp.features(csr.rowptr, csr.col, csr.val, v)
    pos, src, dst, p = mlp.edges(csr.rowptr, csr.col, csr.val)
    rng = np.random.default_rng(seed + 1)
    params = rng.normal(0, 0.3, mlp.NPARAM)
    tgt = rng.normal(0, 1.0, len(src))
    return csr, v, f, src, dst, p, params, tgt


def test_parameter_count():
    assert mlp.NPARAM == 4801


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).normal(0, 10, 100_000).astype(np.float32)
    x[:4] = [1.0, 1.00390625, 1.0078125 + 2**-9, -3.5]      # ties and exact values
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_features_brute_force():
    csr, v, f, *_ = _problem(2, 12)
    n = csr.n
    deg = np.zeros(n)
    r = np.zeros(n)
    nbrs = [[] for _ in range(n)]
    for i in range(n):
        for p in range(csr.rowptr[i], csr.rowptr[i + 1]):
            j, a = csr.col[p], csr.val[p]
            if j != i and a > 0:
                deg[i] += 1
                r[i] += a
                nbrs[i].append(j)
    raw = np.zeros((n, 4))
    for i in range(n):
        mnb = np.mean([deg[j] for j in nbrs[i]]) if nbrs[i] else 0.0
        raw[i] = [np.log1p(deg[i]), r[i], v[i], np.log1p(mnb)]
    exp = (raw - raw.mean(0)) / np.where(raw.std(0) > 0, raw.std(0), 1.0)
    assert np.allclose(f, exp, rtol=1e-13, atol=1e-13)


def test_gradient_matches_finite_differences():
    _, _, f, src, dst, p, params, tgt = _problem(3)
    loss, g = mlp.loss_and_grad(params, f, src, dst, p, tgt, bf=False)
    rng = np.random.default_rng(5)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 600]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        lp, _ = mlp.loss_and_grad(params + e, f, src, dst, p, tgt, bf=False)
        lm, _ = mlp.loss_and_grad(params - e, f, src, dst, p, tgt, bf=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_gradient_matches_torch_autograd():
    _, _, f, src, dst, p, params, tgt = _problem(4)
    loss, g = mlp.loss_and_grad(params, f, src, dst, p, tgt, bf=False)
    pt = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    o = 0
    w1 = pt[o:o + 512].view(64, 8); o += 512
    b1 = pt[o:o + 64]; o += 64
    w2 = pt[o:o + 4096].view(64, 64); o += 4096
    b2 = pt[o:o + 64]; o += 64
    w3 = pt[o:o + 64]; o += 64
    b3 = pt[o]
    ft = torch.tensor(f)
    x = torch.cat([ft[src], ft[dst]], 1)
    y = torch.relu(torch.relu(x @ w1.T + b1) @ w2.T + b2) @ w3 + b3
    b = 8 * torch.tanh(y / 8)
    pw = torch.tensor(p)
    lt = (pw * (b - torch.tensor(tgt)) ** 2).sum() / pw.sum()
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12 * max(1, loss)
    assert np.allclose(pt.grad.numpy(), g, rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=100)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(100), np.zeros(100)
    for step in range(1, 6):
        g = rng.normal(size=100)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam(p, m, v, g, step, 1e-2)
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_targets_for_exact_statistics():
    est = np.array([1.0, 2.0, 4.0])
    se = np.zeros(3)
    src = np.array([0, 1, 2])
    dst = np.array([1, 2, 0])
    t = mlp.targets_from_stats(est, se, 100, src, dst)
    assert np.allclose(t, np.log(est[dst]) - np.log(est[src]), rtol=1e-14)


def test_training_reduces_loss():
    _, _, f, src, dst, p, params, tgt = _problem(7)
    tgt = np.tanh(f[dst, 0] - f[src, 0])        # learnable target
    params = np.random.default_rng(8).normal(0, 0.1, mlp.NPARAM)
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    l0, _ = mlp.loss_and_grad(params, f, src, dst, p, tgt)
    for step in range(1, 201):
        _, g = mlp.loss_and_grad(params, f, src, dst, p, tgt)
        params, m, v = mlp.adam(params, m, v, g, step, 3e-3)
    l1, _ = mlp.loss_and_grad(params, f, src, dst, p, tgt)
    assert l1 < 0.1 * l0


def _two_edge_case():
    """Two nodes, edges 0 -> 1 and 1 -> 0, weights exactly representable (also in
    bfloat16), only a few hidden units active, so that every value can be worked
    out by hand (see test_two_edge_hand_worked)."""
    feats = np.array([[1.0, 0.0, 0.5, -1.0], [0.0, 2.0, -0.5, 1.0]])
    src, dst = np.array([0, 1]), np.array([1, 0])
    w1 = np.zeros((64, 8)); b1 = np.zeros(64)
    w2 = np.zeros((64, 64)); b2 = np.zeros(64)
    w3 = np.zeros(64)
    w1[0, 0], w1[0, 4], b1[0] = 1.0, -1.0, 0.5          # z1_0 = f_i0 - f_j0 + 1/2
    w1[1, 1], w1[1, 7], b1[1] = 0.5, 0.25, 0.25         # z1_1 = f_i1/2 + f_j3/4 + 1/4
    w2[0, 0], w2[0, 1], b2[0] = 1.0, -2.0, 0.25         # z2_0 = a1_0 - 2 a1_1 + 1/4
    w2[1, 0], w2[1, 1], b2[1] = 0.5, 1.0, -0.5          # z2_1 = a1_0/2 + a1_1 - 1/2
    b2[2] = 0.125                                       # z2_2 = 1/8
    w3[0], w3[1], w3[2] = 2.0, -1.0, 4.0
    b3 = -0.5
    return mlp.pack(w1, b1, w2, b2, w3, b3), feats, src, dst


@pytest.mark.parametrize("bf", [False, True])
def test_two_edge_hand_worked(bf):
    """Forward values by hand.  Edge 0 (x = [1,0,.5,-1, 0,2,-.5,1]): z1 = (1.5, 0.5, 0...),
    z2 = (0.75, 0.75, 0.125, 0...), y = 1.5 - 0.75 + 0.5 - 0.5 = 0.75.  Edge 1
    (x = [0,2,-.5,1, 1,0,.5,-1]): z1 = (-0.5, 1.0, 0...), a1 = (0, 1, 0...),
    z2 = (-1.75, 0.5, 0.125, 0...), a2 = (0, 0.5, 0.125, 0...), y = -0.5 + 0.5 - 0.5 = -0.5.
    b = 8 tanh(y / 8).  Every value is a bfloat16, so the rounded network agrees."""
    p, feats, src, dst = _two_edge_case()
    b, (x, z1, a1q, z2, a2, th, _) = mlp.forward(p, feats, src, dst, bf=bf)
    z1e = np.zeros((2, 64)); z1e[0, :2] = [1.5, 0.5]; z1e[1, :2] = [-0.5, 1.0]
    z2e = np.zeros((2, 64)); z2e[0, :3] = [0.75, 0.75, 0.125]; z2e[1, :3] = [-1.75, 0.5, 0.125]
    np.testing.assert_array_equal(z1, z1e)
    np.testing.assert_array_equal(a1q, np.maximum(z1e, 0))
    np.testing.assert_array_equal(z2, z2e)
    np.testing.assert_array_equal(a2, np.maximum(z2e, 0))
    y = np.array([0.75, -0.5])
    np.testing.assert_allclose(b, 8.0 * np.tanh(y / 8.0), rtol=1e-15, atol=0)
    assert b[0] > 0 > b[1]


def test_two_edge_loss_and_gradient_hand_worked():
    """Loss and all 4801 gradient elements by hand, with p = (1/4, 3/4) (sum 1) and
    targets b* = (1/2, -1).  With g_e = 2 p_e (b_e - b*_e)(1 - tanh^2(y_e/8)):
    dz2 of edge 0 = g_0 (2, -1, 4) (units 0-2 active), of edge 1 = g_1 (0, -1, 4)
    (unit 0 inactive); dz1 of edge 0 = (1.5 g_0, -5 g_0), of edge 1 = (0, -g_1)
    (unit 0 inactive there).  Everything else is zero."""
    p, feats, src, dst = _two_edge_case()
    pw = np.array([0.25, 0.75])
    tgt = np.array([0.5, -1.0])
    loss, g = mlp.loss_and_grad(p, feats, src, dst, pw, tgt, bf=False)
    th = np.tanh(np.array([0.75, -0.5]) / 8.0)
    b = 8.0 * th
    d = b - tgt
    assert abs(loss - (0.25 * d[0] ** 2 + 0.75 * d[1] ** 2)) < 1e-15
    g0, g1 = 2.0 * pw * d * (1.0 - th * th)
    x0 = np.array([1.0, 0.0, 0.5, -1.0, 0.0, 2.0, -0.5, 1.0])
    x1 = np.array([0.0, 2.0, -0.5, 1.0, 1.0, 0.0, 0.5, -1.0])
    gw1 = np.zeros((64, 8)); gb1 = np.zeros(64)
    gw2 = np.zeros((64, 64)); gb2 = np.zeros(64); gw3 = np.zeros(64)
    gw1[0] = 1.5 * g0 * x0
    gw1[1] = -5.0 * g0 * x0 - g1 * x1
    gb1[0], gb1[1] = 1.5 * g0, -5.0 * g0 - g1
    gw2[0, 0], gw2[0, 1] = 3.0 * g0, g0                 # dz2_0 = 2 g_0 (edge 0 only)
    gw2[1, 0], gw2[1, 1] = -1.5 * g0, -0.5 * g0 - g1    # dz2_1 = (-g_0, -g_1)
    gw2[2, 0], gw2[2, 1] = 6.0 * g0, 2.0 * g0 + 4.0 * g1
    gb2[0], gb2[1], gb2[2] = 2.0 * g0, -g0 - g1, 4.0 * (g0 + g1)
    gw3[0], gw3[1], gw3[2] = 0.75 * g0, 0.75 * g0 + 0.5 * g1, 0.125 * (g0 + g1)
    expect = mlp.pack(gw1, gb1, gw2, gb2, gw3, g0 + g1)
    np.testing.assert_allclose(g, expect, rtol=1e-14, atol=1e-16)
