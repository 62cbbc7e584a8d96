"""Pins of the FP64 surrogate oracle (CPU only): gradients against central
finite differences and against torch autograd, Adam against torch.optim.Adam,
bfloat16 rounding against torch's conversion, and the ensemble spread rule."""
import numpy as np
import pytest
import torch

from oracle import mlp as M

SMALL = (36, 16, 16, 16, 12)


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 36)), rng.normal(size=(n, 12))


def test_P11_gradients_vs_central_differences():
    Ws, bs = M.init_params(1, SMALL)
    x, t = _data(7)
    _, dWs, dbs = M.backward(Ws, bs, x, t)
    rng = np.random.default_rng(2)
    h = 1e-6
    for l in range(4):
        for _ in range(6):
            i = rng.integers(Ws[l].shape[0]); j = rng.integers(Ws[l].shape[1])
            old = Ws[l][i, j]
            Ws[l][i, j] = old + h; lp = M.mse(M.forward(Ws, bs, x)[0], t)
            Ws[l][i, j] = old - h; lm = M.mse(M.forward(Ws, bs, x)[0], t)
            Ws[l][i, j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dWs[l][i, j]) <= 1e-7 * max(1.0, abs(fd))
        i = rng.integers(bs[l].shape[0])
        old = bs[l][i]
        bs[l][i] = old + h; lp = M.mse(M.forward(Ws, bs, x)[0], t)
        bs[l][i] = old - h; lm = M.mse(M.forward(Ws, bs, x)[0], t)
        bs[l][i] = old
        assert abs((lp - lm) / (2 * h) - dbs[l][i]) <= 1e-7


def test_gradients_vs_torch_autograd_full_size():
    Ws, bs = M.init_params(3)
    for l in range(4):
        bs[l] = np.random.default_rng(10 + l).normal(size=bs[l].shape) * 0.1
    x, t = _data(33, 4)
    loss, dWs, dbs = M.backward(Ws, bs, x, t)
    tW = [torch.tensor(w, requires_grad=True) for w in Ws]
    tb = [torch.tensor(b, requires_grad=True) for b in bs]
    h = torch.tensor(x)
    for l in range(4):
        h = h @ tW[l].T + tb[l]
        if l < 3:
            h = torch.relu(h)
    tl = ((h - torch.tensor(t)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12 * abs(loss)
    for l in range(4):
        np.testing.assert_allclose(dWs[l], tW[l].grad.numpy(), rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(dbs[l], tb[l].grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_vs_torch():
    rng = np.random.default_rng(0)
    p = [rng.normal(size=(5, 4)), rng.normal(size=4)]
    tp = [torch.tensor(a.copy(), requires_grad=True) for a in p]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    mine = M.Adam(p, lr=1e-3)
    for k in range(5):
        g = [rng.normal(size=a.shape) for a in p]
        for a, ga in zip(tp, g):
            a.grad = torch.tensor(ga)
        opt.step()
        mine.step(p, g)
    for a, ta in zip(p, tp):
        np.testing.assert_allclose(a, ta.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_rounding_matches_torch():
    v = np.random.default_rng(1).normal(size=10000) * 10.0 ** np.random.default_rng(2).uniform(-5, 5, 10000)
    v = np.concatenate([v, [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]])
    mine = M.bf16_round(v)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mine, ref)


def test_ensemble_spread_rule():
    Ws, bs = M.init_params(5, SMALL)
    members = [(Ws, bs)] * 4
    feat = np.random.default_rng(0).normal(size=(9, 36))
    z36, o36 = np.zeros(36), np.ones(36)
    r, s, flag = M.ensemble_predict(members, feat, z36, o36, np.full(12, 3.0), np.ones(12))
    assert np.all(s == 0) and not flag.any()
    W2 = [w.copy() for w in Ws]; W2[3] = W2[3] * 1.5
    r, s, flag = M.ensemble_predict([(Ws, bs)] * 3 + [(W2, bs)], feat, z36, o36,
                                    np.zeros(12), np.ones(12), tol=0.05)
    y1 = M.forward(Ws, bs, feat)[0]; y2 = M.forward(W2, bs, feat)[0]
    mean = 0.75 * y1 + 0.25 * y2
    std = np.sqrt(0.75 * (y1 - mean) ** 2 + 0.25 * (y2 - mean) ** 2)
    np.testing.assert_allclose(r, mean, rtol=1e-12)
    np.testing.assert_allclose(s, np.linalg.norm(std, axis=1) / np.linalg.norm(mean, axis=1), rtol=1e-12)
    assert flag.any()
