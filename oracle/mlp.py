"""FP64 NumPy oracle of the slip-rate surrogate -- TEST INFRASTRUCTURE ONLY.

A 4-member ensemble of multilayer perceptrons 36 -> 256 -> 256 -> 256 -> 12
(ReLU on the hidden layers, linear output) maps, per material point, the
resolved shear stress and the mobile and sessile line densities of the 12 FCC
slip systems to the 12 burst-averaged slip rates (the running averages of
Eq. R_lambda_t).  The surrogate is not in the paper; its architecture,
ensemble size, loss and optimiser are fixed by the workload definition, and the
readings taken where that definition is silent are:

* inputs are standardised inside the model: x' = (x - in_shift) * in_scale;
* outputs are standardised targets: rate = y' * out_scale + out_shift;
* loss: mean squared error over batch and outputs in standardised units;
* optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on FP32
  master weights;
* ensemble prediction: the member mean; spread = ||std over members||_2 /
  max(||mean||_2, floor), population std; a point needs DD when spread > tol.

Everything here is written out with NumPy matrix products in float64.
``bf16=True`` rounds the places the device keeps in bfloat16 (weights, layer
inputs) to bfloat16 (round to nearest even) first, so that the comparison with
the device measures accumulation order only.
"""
from __future__ import annotations

import numpy as np

LAYERS = (36, 256, 256, 256, 12)
N_MEMBERS = 4


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the top 16 bits of the IEEE float32 pattern."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int, layers=LAYERS):
    """He-uniform weights, zero biases, float64.  W[l] has shape [out][in]."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for fin, fout in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / fin)
        Ws.append(rng.uniform(-lim, lim, (fout, fin)))
        bs.append(np.zeros(fout))
    return Ws, bs


def forward(Ws, bs, x, bf16=False):
    """x [n][36] standardised inputs -> (y [n][12], cache)."""
    rd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    h = rd(x)
    cache = [h]
    pre = []
    L = len(Ws)
    for l in range(L):
        z = h @ rd(Ws[l]).T + bs[l]
        pre.append(z)
        if l < L - 1:
            h = rd(np.maximum(z, 0.0))
            cache.append(h)
        else:
            h = z
    return h, (cache, pre)


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(Ws, bs, x, t, bf16=False):
    """Gradients of the MSE loss; returns (loss, dWs, dbs)."""
    y, (hs, pre) = forward(Ws, bs, x, bf16)
    rd = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    n, k = y.shape
    g = 2.0 * (y - t) / (n * k)            # dL/dy
    dWs = [None] * len(Ws)
    dbs = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dWs[l] = g.T @ hs[l]
        dbs[l] = g.sum(0)
        if l > 0:
            g = (g @ rd(Ws[l])) * (pre[l - 1] > 0.0)
    return mse(y, t), dWs, dbs


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def transform_features(feat, log_dens=None):
    """Density features 12..35 -> log10(rho * scale + floor) when log_dens =
    (scale, floor) is given; resolved shear stresses unchanged."""
    f = np.array(feat, np.float64)
    if log_dens is not None and log_dens[1] > 0:
        f[:, 12:] = np.log10(np.maximum(f[:, 12:], 0.0) * log_dens[0] + log_dens[1])
    return f


def ensemble_predict(members, feat, in_shift, in_scale, out_shift, out_scale,
                     tol=0.05, floor=1e-30, bf16=False, log_dens=None):
    """members: list of (Ws, bs).  Returns (rates [n][12], spread [n], needs_dd [n])."""
    x = (transform_features(feat, log_dens) - in_shift) * in_scale
    ys = []
    for Ws, bs in members:
        y, _ = forward(Ws, bs, x, bf16)
        ys.append(y * out_scale + out_shift)
    Y = np.stack(ys)                      # [M][n][12]
    mean = Y.mean(0)
    std = np.sqrt(((Y - mean) ** 2).mean(0))
    spread = np.linalg.norm(std, axis=1) / np.maximum(np.linalg.norm(mean, axis=1), floor)
    return mean, spread, spread > tol
