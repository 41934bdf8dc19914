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
