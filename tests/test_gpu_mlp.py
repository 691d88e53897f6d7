"""Learned estimator kernels against the CPU oracle (oracle/mlp.py), and the
gain of the trained network over the closed form."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp
from helpers import to_dev

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
    import torch
    from paper_1910_04658_amd import binding as bs
    rng = np.random.default_rng(N)
    n = 3001  # ragged: not a multiple of the 16-pair tile
    xa, xb, xab = _counts(rng, n, N)
    theta = _theta(rng)
    got = bs.mlp_forward(_w_bf16(theta, dev), to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev), N)
    torch.cuda.synchronize()
    p, _ = mlp.forward(theta, xa, xb, xab, N)
    ref = np.clip(p, 0, 1)
    err = np.abs(got.cpu().numpy() - ref)
    # FP32 accumulation against FP64: ~1e-6; a BF16 rounding of h1 that falls
    # the other way moves one pair by at most ~1e-2
    assert np.quantile(err, 0.99) < 1e-4 and err.max() < 2e-2, (np.quantile(err, 0.99), err.max())


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


@pytest.mark.parametrize("n", [4096, 1000])
def test_gradient_matches_oracle(n, dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    N = 256
    rng = np.random.default_rng(n)
    xa, xb, xab = _counts(rng, n, N)
    label = rng.random(n).astype(np.float32)
    theta = _theta(rng)
    g, loss = bs.mlp_grad(_w_bf16(theta, dev), to_dev(xa, dev), to_dev(xb, dev), to_dev(xab, dev),
                          to_dev(label, dev), N)
    torch.cuda.synchronize()
    lref, gref = mlp.loss_and_grad(theta, xa, xb, xab, label.astype(np.float64), N)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - lref) <= 1e-5 * lref
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert rel < 2e-3, rel
    for name, sl in mlp.SLICES.items():
        r = np.linalg.norm(g[sl] - gref[sl]) / max(np.linalg.norm(gref[sl]), 1e-12)
        assert r < 1e-2, (name, r)


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
    _, gref = mlp.loss_and_grad(theta, xa, xb, xab, label.astype(np.float64), N)
    tref, mref, vref = mlp.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), gref, 1, lr)
    got = master.cpu().numpy().astype(np.float64)
    # Adam's first step moves each weight by about lr * sign(g): compare where the
    # gradient is not close to zero (its sign is then unambiguous)
    big = np.abs(gref) > 1e-2 * np.abs(gref).max()
    assert big.sum() > 300
    assert np.max(np.abs(got[big] - tref[big])) < 1e-6
    np.testing.assert_allclose(m.cpu().numpy()[big], mref[big], rtol=2e-2)
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
