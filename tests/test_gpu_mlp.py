"""Learned estimator kernels against the CPU oracle (oracle/mlp.py), and the
gain of the trained network over the closed form."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp
from helpers import to_dev
from mlp_bounds import Bounds

pytestmark = pytest.mark.gpu


def _counts(rng, n, N):
    xa = rng.integers(0, N + 1, n)
    xb = rng.integers(0, N + 1, n)
    lo = np.maximum(0, xa + xb - N)
    hi = np.minimum(xa, xb)
    xab = lo + (rng.random(n) * (hi - lo + 1)).astype(np.int64)
    return xa.astype(np.int32), xb.astype(np.int32), xab.astype(np.int32)


def _theta(rng, scale=0.3):
    t = rng.normal(0, scale, mlp.N_PARAMS)
    t[mlp.SLICES["w3"]] *= 0.3
    return mlp.bf16_round(t)


def _w_bf16(theta, dev):
    import torch
    u = np.asarray(theta, np.float32).view(np.uint32) >> 16
    return torch.from_numpy(u.astype(np.uint16).view(np.int16)).to(dev)


def test_pair_popcount_matches_oracle(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    c = datagen.small_corpus(n=700, d=9000, seed=31)
    N = 512
    pi = datagen.random_map(c.d, N, 31)
    w, _ = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    rng = np.random.default_rng(0)
    ia = rng.integers(0, 700, 5003).astype(np.int32)
    ib = rng.integers(0, 700, 5003).astype(np.int32)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    got = bs.pair_popcount(w, to_dev(ia, dev), w, to_dev(ib, dev), N, err_flag=flag).cpu().numpy()
    S = oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)
    X = oracle.intersections(S, S)
    assert int(flag.item()) == 0
    assert np.array_equal(got, X[ia, ib])


@pytest.mark.parametrize("N", [256, 1024, 192])
def test_forward_matches_oracle(N, dev):
    """Every prediction within the error radius derived for an FP32
    evaluation of the oracle's model (tests/mlp_bounds.py): FP32 rounding of
    each layer, and BF16 roundings of h1 or ReLU decisions that lie within
    that rounding of their boundary taken as flipped. (N = 192 is not a power
    of two: x/N is then rounded, the same IEEE division on both sides.)"""
    import torch
    from paper_1910_04658_amd import binding as bs
    rng = np.random.default_rng(N)
    n = 3001  # ragged: not a multiple of the 16-pair tile
    xa, xb, xab = _counts(rng, n, N)
    theta = _theta(rng)
    got = bs.mlp_forward(_w_bf16(theta, dev), to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev), N)
    torch.cuda.synchronize()
    B = Bounds(theta, xa, xb, xab, np.zeros(n), N)
    err = np.abs(got.cpu().numpy().astype(np.float64) - np.clip(B.p, 0, 1))
    bad = np.nonzero(err > B.p_bound)[0]
    assert len(bad) == 0, (bad[:5], err[bad[:5]], B.p_bound[bad[:5]])


def test_zero_weights_give_the_topk_closed_form(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    N = 256
    rng = np.random.default_rng(7)
    xa, xb, xab = _counts(rng, 777, N)
    zero = torch.zeros(mlp.N_PARAMS, dtype=torch.int16, device=dev)
    got = bs.mlp_forward(zero, to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev), N).cpu().numpy()
    ref = np.clip(mlp.closed_form(xa, xb, xab, N), 0, 1).astype(np.float32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("N,n", [(256, 4096), (256, 1000), (1024, 3001), (512, 20000)])
def test_gradient_matches_oracle(N, n, dev):
    """Every one of the 4,545 gradient entries, and the loss, within the bound
    derived for an FP32 evaluation of the oracle's gradient
    (tests/mlp_bounds.py): 2u (n + 96) times the entry's sum of |terms| for
    FP32 rounding and accumulation over the batch, the absolute error of
    dL/dy carried through, and the first-order effect of any BF16 rounding or
    ReLU decision within its rounding error of the boundary."""
    import torch
    from paper_1910_04658_amd import binding as bs
    rng = np.random.default_rng(n)
    xa, xb, xab = _counts(rng, n, N)
    label = rng.random(n).astype(np.float32)
    theta = _theta(rng)
    g, loss = bs.mlp_grad(_w_bf16(theta, dev), to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev),
                          to_dev(label, dev), N)
    torch.cuda.synchronize()
    B = Bounds(theta, xa, xb, xab, label.astype(np.float64), N)
    assert abs(float(loss.item()) - B.loss) <= B.loss_bound
    d = np.abs(g.cpu().numpy().astype(np.float64) - B.grad)
    bad = np.nonzero(d > B.grad_bound)[0]
    assert len(bad) == 0, (bad[:5], d[bad[:5]], B.grad_bound[bad[:5]], B.grad[bad[:5]])


def test_gradient_is_deterministic(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    N = 512
    rng = np.random.default_rng(11)
    xa, xb, xab = _counts(rng, 20000, N)
    label = rng.random(20000).astype(np.float32)
    w = _w_bf16(_theta(rng), dev)
    args = (to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev), to_dev(label, dev), N)
    g1, l1 = bs.mlp_grad(w, *args)
    g2, l2 = bs.mlp_grad(w, *args)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_train_step_matches_oracle_adam(dev):
    """One Adam step from zero moments moves entry j by lr * g_j / (|g_j| + eps)
    (bias-corrected moments at step 1 are g and g^2). With the GPU gradient
    within its derived bound of the oracle's, an entry whose oracle gradient
    exceeds the bound has a known sign and moves by lr * sign(g) up to
    lr * eps / (|g| - bound); every other entry moves by at most lr. The
    first moment is 0.1 g within 0.1 times the bound; the BF16 copy is the
    rounded master."""
    import torch
    from paper_1910_04658_amd import binding as bs
    N = 256
    rng = np.random.default_rng(12)
    n = 2048
    xa, xb, xab = _counts(rng, n, N)
    label = rng.random(n).astype(np.float32)
    theta = _theta(rng)
    master = torch.from_numpy(theta.astype(np.float32)).to(dev)
    w = _w_bf16(theta, dev)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    lr = 1e-3
    bs.mlp_train_step(master, w, m, v, 1, lr, to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev),
                      to_dev(label, dev), N)
    torch.cuda.synchronize()
    B = Bounds(theta, xa, xb, xab, label.astype(np.float64), N)
    g, gb = B.grad, B.grad_bound
    got = master.cpu().numpy().astype(np.float64)
    u = 2.0 ** -24
    rnd = 8 * u * (np.abs(theta) + lr)
    sure = np.abs(g) > gb
    assert sure.sum() > 0.5 * mlp.N_PARAMS
    want = theta - lr * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8)
    tol = lr * 1e-8 / np.maximum(np.abs(g) - gb, 1e-30) + rnd
    assert np.all(np.abs(got[sure] - want[sure]) <= tol[sure])
    assert np.all(np.abs(got[~sure] - theta[~sure]) <= lr + rnd[~sure])
    mm = m.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(mm - 0.1 * g) <= 0.1 * gb + 8 * u * np.abs(g) + 1e-30)
    wb = w.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(wb.view(np.float32), mlp.bf16_round(master.cpu().numpy()).astype(np.float32))


def test_trained_network_beats_closed_form_at_saturation(dev):
    """Trained on near-duplicate pairs sketched at N = 256 (where long rows
    saturate the sketch), the network's Jaccard MSE on held-out pairs is well
    below the closed form's."""
    from paper_1910_04658_amd import learned
    N = 256
    tr = datagen.variant_groups(500, 16, seed=101)
    te = datagen.variant_groups(200, 16, seed=202)
    pi = datagen.random_map(tr.csr.d, N, 77)
    dtr = learned.sketch_pairs(tr, pi, N, dev)
    dte = learned.sketch_pairs(te, pi, N, dev)
    model = learned.Model(learned.init_master(0, dev))
    model.train(dtr, steps=800, batch=4096, lr=3e-3, seed=0)
    mse_l = learned.mse(model.predict(dte), dte)
    mse_c = learned.mse(learned.closed_form(dte), dte)
    print("held-out MSE: learned %.3e, closed form %.3e" % (mse_l, mse_c))
    assert mse_l < 0.9 * mse_c
