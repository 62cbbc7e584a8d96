"""GPU parity of the BF16-MFMA surrogate kernels against the FP64 NumPy oracle
(forward with the device's bfloat16 rounding points emulated, gradients,
Adam), plus training, ensemble-spread and chunking behaviour.

Tolerances: bfloat16 operands with float32 accumulation against FP64 -> a
normwise relative error of 2e-2 per tensor (rounding of activations and
gradients to 8-bit mantissas, ~4e-3 each, through four layers).
"""
import numpy as np
import pytest
import torch

import paper_2005_02498_amd as dd
from oracle import mlp as M

pytestmark = pytest.mark.gpu
TOL = 2e-2
DEV = torch.device("cuda:0")


def flat(Ws, bs):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)]).astype(np.float32)


def unflat(p):
    out, o = [], 0
    Ws, bs = [], []
    for fin, fout in zip(M.LAYERS[:-1], M.LAYERS[1:]):
        Ws.append(p[o:o + fin * fout].reshape(fout, fin).astype(np.float64)); o += fin * fout
        bs.append(p[o:o + fout].astype(np.float64)); o += fout
    assert o == dd.MLP_PARAMS
    return Ws, bs


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _model(members=4, seed=0, scaling=True):
    mdl = dd.SurrogateModel(members, seed)
    params = []
    for m in range(members):
        Ws, bs = M.init_params(100 + m)
        for l in range(4):
            bs[l] = np.random.default_rng(200 + 10 * m + l).normal(size=bs[l].shape) * 0.05
        p = flat(Ws, bs)
        mdl.set_params(m, p)
        params.append(unflat(p))
    rng = np.random.default_rng(7)
    sc = (rng.normal(size=36).astype(np.float32), rng.uniform(0.5, 2, 36).astype(np.float32),
          rng.normal(size=12).astype(np.float32), rng.uniform(0.5, 2, 12).astype(np.float32))
    if scaling:
        mdl.set_scaling(*sc)
    else:
        sc = (np.zeros(36, np.float32), np.ones(36, np.float32), np.zeros(12, np.float32),
              np.ones(12, np.float32))
    return mdl, params, sc


def test_params_roundtrip():
    mdl, params, _ = _model(2)
    p = mdl.get_params(1)
    np.testing.assert_array_equal(p, flat(*params[1]))


@pytest.mark.parametrize("n", [1, 255, 257, 1000])
def test_forward_parity(n):
    """Against the bf16-emulating oracle; n spans one partial, one full plus one
    row and several 256-row workgroups with a ragged tail."""
    mdl, params, sc = _model()
    feat = np.random.default_rng(1).normal(size=(n, 36)).astype(np.float32)
    r, s, f = dd.dd_surrogate_rates(mdl, torch.tensor(feat, device=DEV), 0.05)
    torch.cuda.synchronize()
    ro, so, fo = M.ensemble_predict(params, feat.astype(np.float64), sc[0], sc[1], sc[2], sc[3],
                                    tol=0.05, bf16=True)
    e = nrel(r.cpu().numpy(), ro)
    print(f"surrogate forward rates err {e:.2e}, spread err {nrel(s.cpu().numpy(), so):.2e}")
    assert e < TOL
    assert nrel(s.cpu().numpy(), so) < TOL
    # exact (unrounded) FP64 network: still within the bfloat16 budget
    ro64, _, _ = M.ensemble_predict(params, feat.astype(np.float64), sc[0], sc[1], sc[2], sc[3])
    assert nrel(r.cpu().numpy(), ro64) < TOL


@pytest.mark.parametrize("n", [1, 37, 1024])
def test_gradient_parity(n):
    mdl, params, sc = _model()
    rng = np.random.default_rng(n)
    feat = rng.normal(size=(n, 36)).astype(np.float32)
    tgt = rng.normal(size=(n, 12)).astype(np.float32)
    g, loss = dd.dd_mlp_gradients(mdl, torch.tensor(feat, device=DEV), torch.tensor(tgt, device=DEV))
    torch.cuda.synchronize()
    g = g.cpu().numpy(); loss = loss.cpu().numpy()
    x = (feat.astype(np.float64) - sc[0]) * sc[1]
    t = (tgt.astype(np.float64) - sc[2]) / sc[3]
    worst = 0.0
    for m in range(4):
        Ws, bs = params[m]
        lo, dWs, dbs = M.backward(Ws, bs, x, t, bf16=True)
        assert abs(loss[m] - lo) / lo < 1e-2
        ref = flat(dWs, dbs).astype(np.float64)
        gw, gb = unflat(g[m])
        for l in range(4):
            worst = max(worst, nrel(gw[l], dWs[l]), nrel(gb[l], dbs[l]))
        worst = max(worst, nrel(g[m], ref))
    print(f"surrogate gradients n={n} worst tensor err {worst:.2e}")
    assert worst < TOL


def test_adam_step_matches_formula():
    mdl, params, sc = _model(2)
    rng = np.random.default_rng(3)
    feat = torch.tensor(rng.normal(size=(256, 36)).astype(np.float32), device=DEV)
    tgt = torch.tensor(rng.normal(size=(256, 12)).astype(np.float32), device=DEV)
    g, _ = dd.dd_mlp_gradients(mdl, feat, tgt)
    g = g.cpu().numpy().astype(np.float64)
    p0 = np.stack([mdl.get_params(m) for m in range(2)]).astype(np.float64)
    lr = 1e-3
    dd.dd_mlp_train_step(mdl, feat, tgt, lr)
    torch.cuda.synchronize()
    p1 = np.stack([mdl.get_params(m) for m in range(2)]).astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2
    exp = p0 - lr * g / (np.abs(g) + 1e-8)
    bound = 2e-6 * lr + 1e-7 * np.abs(p0)
    assert np.all(np.abs(p1 - exp) <= bound), float(np.max(np.abs(p1 - exp) - bound))


def test_training_reduces_loss():
    mdl = dd.SurrogateModel(4, 11)
    rng = np.random.default_rng(0)
    Wt = rng.normal(size=(36, 12)) / 6.0
    X = rng.normal(size=(4096, 36)).astype(np.float32)
    Y = np.tanh(X @ Wt).astype(np.float32) + 0.1 * (X[:, :12] ** 2).astype(np.float32)
    Xd = torch.tensor(X, device=DEV); Yd = torch.tensor(Y, device=DEV)
    first = None
    for it in range(300):
        b = (it * 256) % 4096
        loss = dd.dd_mlp_train_step(mdl, Xd[b:b + 256].contiguous(), Yd[b:b + 256].contiguous(), 1e-3)
        if first is None:
            first = loss.cpu().numpy().copy()
    last = loss.cpu().numpy()
    print(f"training loss {first} -> {last}")
    assert np.all(last < 0.2 * first)


def test_ensemble_spread_and_fallback():
    mdl = dd.SurrogateModel(4, 5)
    Ws, bs = M.init_params(9)
    p = flat(Ws, bs)
    for m in range(4):
        mdl.set_params(m, p)
    mdl.set_scaling(np.zeros(36), np.ones(36), np.full(12, 10.0), np.ones(12))
    feat = torch.tensor(np.random.default_rng(2).normal(size=(500, 36)).astype(np.float32), device=DEV)
    r, s, f = dd.dd_surrogate_rates(mdl, feat, 0.05)
    assert float(s.max()) < 1e-6 and int(f.sum()) == 0
    r, s, f = dd.dd_surrogate_rates(mdl, feat, 0.0)
    assert int(f.sum()) == 0          # spread exactly 0 is not above a zero tolerance
    q = p.copy()
    q[dd.MLP_PARAMS - 12:] += 5.0    # shift one member's output biases
    mdl.set_params(3, q)
    r, s, f = dd.dd_surrogate_rates(mdl, feat, 0.05)
    assert int(f.sum()) == 500


def test_chunked_inference_consistent():
    mdl, params, sc = _model(2)
    n = 262144 + 1000
    feat = torch.tensor(np.random.default_rng(4).normal(size=(n, 36)).astype(np.float32), device=DEV)
    r, s, f = dd.dd_surrogate_rates(mdl, feat, 0.05)
    sl = slice(262144 - 300, 262144 + 300)
    r2, s2, f2 = dd.dd_surrogate_rates(mdl, feat[sl].contiguous(), 0.05)
    np.testing.assert_array_equal(r[sl].cpu().numpy(), r2.cpu().numpy())
    np.testing.assert_array_equal(s[sl].cpu().numpy(), s2.cpu().numpy())


def test_invalid_arguments():
    mdl = dd.SurrogateModel(2, 0)
    f = torch.zeros((70000, 36), dtype=torch.float32, device=DEV)
    t = torch.zeros((70000, 12), dtype=torch.float32, device=DEV)
    with pytest.raises(dd.DDError):
        dd.dd_mlp_train_step(mdl, f, t)
    with pytest.raises(dd.DDError):
        mdl.set_params(2, np.zeros(dd.MLP_PARAMS, np.float32))
    with pytest.raises(dd.DDError):
        dd.SurrogateModel(0, 0)


def test_forward_parity_log_densities():
    mdl, params, sc = _model()
    rng = np.random.default_rng(5)
    feat = np.concatenate([rng.normal(size=(300, 12)) * 5e7,
                           np.where(rng.uniform(size=(300, 24)) < 0.3, 0.0,
                                    10 ** rng.uniform(-9, -6, (300, 24)))], 1).astype(np.float32)
    dens = (1.0 / (0.2556e-9) ** 2, 1e10)
    mdl.set_log_densities(*dens)
    shift = np.concatenate([np.zeros(12), np.full(24, 12.0)]).astype(np.float32)
    scale = np.concatenate([np.full(12, 1e-8), np.full(24, 1.0)]).astype(np.float32)
    mdl.set_scaling(shift, scale, sc[2], sc[3])
    r, s, f = dd.dd_surrogate_rates(mdl, torch.tensor(feat, device=DEV), 0.05)
    ro, so, fo = M.ensemble_predict(params, feat.astype(np.float64), shift, scale, sc[2], sc[3],
                                    tol=0.05, bf16=True, log_dens=dens)
    e = nrel(r.cpu().numpy(), ro)
    print(f"surrogate forward with log densities err {e:.2e}")
    assert e < TOL
