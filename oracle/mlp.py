"""Learned Jaccard estimator — CPU oracle (TEST INFRASTRUCTURE ONLY).

A 4 -> 64 -> 64 -> 1 ReLU network that corrects the closed-form Jaccard
estimate of Algorithm 3 where sketches saturate. Its inputs are the three
sketch counts of Algorithm 1 (|a_s|, |b_s|, |a_s AND b_s|) and the width N; the
paper has no such network — it is an extension built on the paper's
estimator, which stays the baseline it is judged against.

Model (the definition the GPU kernels follow, evaluated here in FP64):
  f   = (x_a/N, x_b/N, x_ab/N, log2(N)/16)                        features
  z1  = W1 f + b1,  h1 = relu(z1)                                 64 units
  z2  = W2 bf16(h1) + b2,  h2 = relu(z2)                          64 units
  y   = w3 . h2 + b3
  p   = JS_closed(x_a, x_b, x_ab, N) + y                          prediction
with the FP32 closed form of Algorithms 1-3 (oracle.score_f32, measure JS).
Loss over a batch of n pairs with exact Jaccard labels t: mean (p - t)^2.
Gradients by hand-written backpropagation; where the GPU rounds an operand of
its BF16 matrix products (h1 for layer 2 and for dW2, and dz2 for dW2 and dh1)
this oracle applies the same round-to-nearest-even to BF16 (bf16=True), so the
two sides differ only by FP32 accumulation order. With bf16=False the model is
smooth and its gradients are pinned by finite differences.

Parameters are one flat float64 vector of 4,545 entries, in this order:
W1[64][4], b1[64], W2[64][64] (row = output unit), b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

H = 64
N_PARAMS = H * 4 + H + H * H + H + H + 1  # 4545
SLICES = {}
_o = 0
for _name, _size in (("W1", H * 4), ("b1", H), ("W2", H * H), ("b2", H), ("w3", H), ("b3", 1)):
    SLICES[_name] = slice(_o, _o + _size)
    _o += _size
assert _o == N_PARAMS


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    return {"W1": theta[SLICES["W1"]].reshape(H, 4), "b1": theta[SLICES["b1"]],
            "W2": theta[SLICES["W2"]].reshape(H, H), "b2": theta[SLICES["b2"]],
            "w3": theta[SLICES["w3"]], "b3": theta[SLICES["b3"]][0]}


def pack(g):
    return np.concatenate([np.ravel(g["W1"]), g["b1"], np.ravel(g["W2"]), g["b2"], g["w3"],
                           np.atleast_1d(g["b3"])]).astype(np.float64)


def bf16_round(x):
    """Round float values to the nearest BF16 value (ties to even), via their
    FP32 bit patterns: keep the top 16 bits after adding 0x7FFF + lsb."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def features(xa, xb, xab, N):
    xa = np.asarray(xa, np.float32)
    Nf = np.float32(N)
    f = np.stack([xa / Nf, np.asarray(xb, np.float32) / Nf, np.asarray(xab, np.float32) / Nf,
                  np.full(xa.shape, np.float32(np.log2(float(N)) / 16.0))], axis=1)
    return f.astype(np.float64)


def closed_form(xa, xb, xab, N):
    from . import JS, score_f32
    return np.array([float(score_f32(a, b, c, N, JS)) for a, b, c in zip(xa, xb, xab)], np.float64)


def forward(theta, xa, xb, xab, N, bf16=True, base=None):
    """Returns (prediction p, cache) for pairs given by their sketch counts."""
    P = unpack(theta)
    f = features(xa, xb, xab, N)
    if base is None:
        base = closed_form(xa, xb, xab, N)
    z1 = f @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    h1q = bf16_round(h1) if bf16 else h1
    z2 = h1q @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["w3"] + P["b3"]
    p = base + y
    return p, {"f": f, "z1": z1, "h1q": h1q, "z2": z2, "h2": h2, "base": base}


def loss_and_grad(theta, xa, xb, xab, label, N, bf16=True, base=None):
    """Mean squared error over the batch and its gradient (flat, FP64)."""
    P = unpack(theta)
    p, c = forward(theta, xa, xb, xab, N, bf16=bf16, base=base)
    n = len(p)
    r = p - np.asarray(label, np.float64)
    loss = float(np.mean(r * r))
    gy = 2.0 * r / n                                   # dL/dy per pair
    g = {"b3": np.sum(gy), "w3": c["h2"].T @ gy}
    gz2 = np.outer(gy, P["w3"]) * (c["z2"] > 0)        # [n][64]
    g["b2"] = gz2.sum(0)
    gz2q = bf16_round(gz2) if bf16 else gz2
    g["W2"] = gz2q.T @ c["h1q"]                         # [out][in]
    gh1 = gz2q @ P["W2"]                               # [n][in]
    gz1 = gh1 * (c["z1"] > 0)
    g["b1"] = gz1.sum(0)
    g["W1"] = gz1.T @ c["f"]
    return loss, pack(g)


def init_params(seed: int = 0):
    """He-uniform initialisation, rounded to BF16, and a zero output layer so
    the untrained network returns the closed form exactly."""
    rng = np.random.default_rng(seed)
    g = {"W1": rng.uniform(-1, 1, (H, 4)) * np.sqrt(6.0 / 4), "b1": np.zeros(H),
         "W2": rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H), "b2": np.zeros(H),
         "w3": np.zeros(H), "b3": 0.0}
    return bf16_round(pack(g))


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) of the FP32 master weights."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
