"""Pins of the learned-estimator oracle (oracle/mlp.py): gradients against
finite differences, BF16 rounding against torch's bfloat16 conversion, the
forward pass against an explicit loop, Adam against torch.optim.Adam."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def _counts(rng, n, N):
    xa = rng.integers(0, N + 1, n)
    xb = rng.integers(0, N + 1, n)
    xab = np.array([rng.integers(max(0, a + b - N), min(a, b) + 1) for a, b in zip(xa, xb)])
    return xa, xb, xab


def _random_theta(rng, scale=0.5):
    return mlp.bf16_round(rng.normal(0, scale, mlp.N_PARAMS))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    N = 256
    xa, xb, xab = _counts(rng, 40, N)
    label = rng.random(40)
    theta = rng.normal(0, 0.4, mlp.N_PARAMS)
    base = mlp.closed_form(xa, xb, xab, N)
    loss, g = mlp.loss_and_grad(theta, xa, xb, xab, label, N, bf16=False, base=base)
    eps = 1e-6
    idx = list(range(0, 256, 17)) + list(range(256, 320, 7)) + list(range(320, 4416, 131)) + \
        list(range(4416, 4545, 5)) + [4544]
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp, _ = mlp.loss_and_grad(tp, xa, xb, xab, label, N, bf16=False, base=base)
        lm, _ = mlp.loss_and_grad(tm, xa, xb, xab, label, N, bf16=False, base=base)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-5, 1000), [0.0, -0.0, 1.0, 1 + 2 ** -8,
                        1 + 3 * 2 ** -9, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(x).astype(np.float32), ref)


def test_forward_against_explicit_loop():
    rng = np.random.default_rng(2)
    N = 1024
    xa, xb, xab = _counts(rng, 12, N)
    theta = _random_theta(rng)
    P = mlp.unpack(theta)
    p, _ = mlp.forward(theta, xa, xb, xab, N, bf16=False)
    for k in range(12):
        f = [xa[k] / N, xb[k] / N, xab[k] / N, np.log2(N) / 16]
        h1 = [max(0.0, sum(P["W1"][u][c] * f[c] for c in range(4)) + P["b1"][u]) for u in range(64)]
        h2 = [max(0.0, sum(P["W2"][o][i] * h1[i] for i in range(64)) + P["b2"][o]) for o in range(64)]
        y = sum(P["w3"][o] * h2[o] for o in range(64)) + P["b3"]
        base = float(oracle.score_f32(xa[k], xb[k], xab[k], N, oracle.JS))
        assert abs(p[k] - (base + y)) < 1e-9


def test_zero_output_layer_is_the_closed_form():
    rng = np.random.default_rng(3)
    N = 256
    xa, xb, xab = _counts(rng, 50, N)
    theta = mlp.init_params(3)
    p, _ = mlp.forward(theta, xa, xb, xab, N)
    assert np.array_equal(p, mlp.closed_form(xa, xb, xab, N))


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    theta = rng.normal(0, 1, 100)
    m = np.zeros(100)
    v = np.zeros(100)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(0, 1, 100)
        theta, m, v = mlp.adam_step(theta, m, v, g, step, 1e-2)
        opt.zero_grad()
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(theta, t.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_bf16_gradient_against_autograd():
    """The BF16 path of the oracle's hand-written backpropagation against
    torch autograd in FP64 on the CPU, with the roundings written as
    straight-through steps: h1 is rounded to BF16 on the way forward (its
    gradient passes unchanged), and the gradient reaching the layer-2 product
    from z2 is rounded to BF16 on the way back (b2 takes it unrounded). That
    is the model the rounding points define; autograd differentiates it
    independently of the oracle's own chain rule."""
    torch = pytest.importorskip("torch")

    def bf16(t):
        return torch.from_numpy(mlp.bf16_round(t.detach().numpy()))

    class RoundForward(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return bf16(x)

        @staticmethod
        def backward(ctx, g):
            return g

    class RoundBackward(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return x.clone()

        @staticmethod
        def backward(ctx, g):
            return bf16(g)

    rng = np.random.default_rng(6)
    N = 256
    xa, xb, xab = _counts(rng, 300, N)
    label = rng.random(300)
    theta = _random_theta(rng, 0.4)
    base = mlp.closed_form(xa, xb, xab, N)
    loss, g = mlp.loss_and_grad(theta, xa, xb, xab, label, N, bf16=True, base=base)
    P = {k: torch.tensor(np.array(v, np.float64), requires_grad=True) for k, v in mlp.unpack(theta).items()}
    f = torch.from_numpy(mlp.features(xa, xb, xab, N))
    z1 = f @ P["W1"].T + P["b1"]
    h1q = RoundForward.apply(torch.relu(z1))
    z2 = RoundBackward.apply(h1q @ P["W2"].T) + P["b2"]
    y = torch.relu(z2) @ P["w3"] + P["b3"]
    p = torch.from_numpy(base) + y
    L = torch.mean((p - torch.from_numpy(label)) ** 2)
    L.backward()
    ref = mlp.pack({k: v.grad.numpy() for k, v in P.items()})
    assert abs(float(L) - loss) <= 1e-12 * loss
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    # the rounding matters: the smooth model's gradient differs
    _, g_smooth = mlp.loss_and_grad(theta, xa, xb, xab, label, N, bf16=False, base=base)
    assert np.abs(g_smooth - ref).max() > 1e-6 * np.abs(ref).max()
