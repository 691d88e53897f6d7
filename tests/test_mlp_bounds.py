"""The derived error bounds of tests/mlp_bounds.py (used by the GPU tests of
the learned estimator) against an independent FP32 evaluation of the same
model on the CPU: numpy float32 arithmetic, with its own summation order
(BLAS blocking), BF16 roundings at the same points. Each entry must fall
within its bound, and the bounds must be tight enough to mean something."""
import numpy as np
import pytest

from oracle import mlp
from mlp_bounds import Bounds


def _counts(rng, n, N):
    xa = rng.integers(0, N + 1, n)
    xb = rng.integers(0, N + 1, n)
    lo = np.maximum(0, xa + xb - N)
    hi = np.minimum(xa, xb)
    xab = lo + (rng.random(n) * (hi - lo + 1)).astype(np.int64)
    return xa.astype(np.int32), xb.astype(np.int32), xab.astype(np.int32)


def _fp32_model(theta, xa, xb, xab, label, N):
    """Forward, loss and gradient in float32 with BF16 roundings of h1 and of
    dz2 (for dW2 and dh1)."""
    P = {k: np.asarray(v, np.float32) for k, v in mlp.unpack(theta).items()}
    f = mlp.features(xa, xb, xab, N).astype(np.float32)
    base = mlp.closed_form(xa, xb, xab, N).astype(np.float32)

    def bf(x):
        return mlp.bf16_round(x).astype(np.float32)

    z1 = f @ P["W1"].T + P["b1"]
    h1q = bf(np.maximum(z1, 0))
    z2 = h1q @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0)
    p = base + (h2 @ P["w3"] + np.float32(P["b3"]))
    n = len(xa)
    r = p - label.astype(np.float32)
    gy = np.float32(2) * r / np.float32(n)
    g = {"b3": gy.sum(), "w3": h2.T @ gy}
    gz2 = np.outer(gy, P["w3"]) * (z2 > 0)
    g["b2"] = gz2.sum(0)
    gz2q = bf(gz2)
    g["W2"] = gz2q.T @ h1q
    gz1 = (gz2q @ P["W2"]) * (z1 > 0)
    g["b1"] = gz1.sum(0)
    g["W1"] = gz1.T @ f
    loss = float(np.mean(r.astype(np.float64) ** 2))
    return p.astype(np.float64), loss, mlp.pack({k: np.asarray(v, np.float64) for k, v in g.items()})


@pytest.mark.parametrize("N,n,seed", [(256, 4096, 1), (256, 1000, 2), (1024, 3001, 3), (512, 20000, 4)])
def test_bounds_cover_an_fp32_evaluation(N, n, seed):
    rng = np.random.default_rng(seed)
    xa, xb, xab = _counts(rng, n, N)
    label = rng.random(n)
    t = rng.normal(0, 0.3, mlp.N_PARAMS)
    t[mlp.SLICES["w3"]] *= 0.3
    theta = mlp.bf16_round(t)
    B = Bounds(theta, xa, xb, xab, label, N)
    p, loss, g = _fp32_model(theta, xa, xb, xab, label, N)
    assert np.all(np.abs(p - B.p) <= B.p_bound)
    assert abs(loss - B.loss) <= B.loss_bound
    assert np.all(np.abs(g - B.grad) <= B.grad_bound)
    # not vacuous: most entries are bounded to well under 1% of their size
    live = np.abs(B.grad) > 0
    assert np.median(B.grad_bound[live] / np.abs(B.grad[live])) < 1e-2
    assert np.median(B.p_bound) < 1e-3
