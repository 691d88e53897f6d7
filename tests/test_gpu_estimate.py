"""bs_and_popcount (bit-exact) and bs_estimate (FP64, 1e-6 relative) against
the CPU oracle."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import sets_rows, to_dev

pytestmark = pytest.mark.gpu

RTOL = 1e-6  # |gpu - oracle| <= RTOL * max(|oracle|, 1)


def sketches(c, N, seed, dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    pi = datagen.random_map(c.d, N, seed)
    w, _ = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    torch.cuda.synchronize()
    S = oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)
    return w, S


def check_pairs(wA, SA, wB, SB, N):
    import torch
    from paper_1910_04658_amd import binding as bs
    X = oracle.intersections(SA, SB)
    gx = bs.and_popcount(wA, wB, N)
    est = bs.estimate(wA, wB, N)
    torch.cuda.synchronize()
    assert np.array_equal(gx.cpu().numpy(), X)
    ref = oracle.estimate_pairs(SA.length, SB.length, X, N)
    for m, key in enumerate(["ip", "ham", "js", "cos"]):
        got = est[key].cpu().numpy()
        err = np.abs(got - ref[m]) / np.maximum(np.abs(ref[m]), 1.0)
        assert err.max() <= RTOL, "%s: max scaled error %g" % (key, err.max())


def test_all_pairs_small_corpus(dev):
    """All 1,000 x 1,000 estimates (diagonal included) at N = 1024."""
    c = datagen.small_corpus()
    w, S = sketches(c, 1024, datagen.SEED_PI, dev)
    check_pairs(w, S, w, S, 1024)


@pytest.mark.parametrize("N", [64, 128, 192, 256, 640, 2048, 4096, 8192])
def test_widths_and_ragged_shapes(N, dev):
    c = datagen.small_corpus(n=517, d=8000, seed=N)
    w, S = sketches(c, N, N, dev)
    a = np.arange(0, 517, 3)[:131]
    b = np.arange(517)
    check_pairs(w[a.tolist()].contiguous(), sets_rows(S, a), w, S, N)


def test_saturated_and_empty_sketches(dev):
    """Rows that fill every bit (x = N), rows that fill all but one, and empty rows."""
    N = 64
    d = 4096
    rng = np.random.default_rng(2)
    rows = [list(range(d)), list(range(d)), [], [5], list(rng.integers(0, d, 40)), list(range(0, d, 2))]
    c = datagen.from_rows(rows, d)
    pi = np.arange(d, dtype=np.int32) % N
    pi[0] = 0
    import torch
    from paper_1910_04658_amd import binding as bs
    w, _ = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    torch.cuda.synchronize()
    S = oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)
    assert S.length[0] == N
    check_pairs(w, S, w, S, N)
    est = bs.estimate(w, w, N)
    for key in est:
        assert torch.isfinite(est[key]).all()


def test_one_by_one_and_empty(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    c = datagen.small_corpus(n=3, d=500, seed=1)
    w, S = sketches(c, 128, 3, dev)
    check_pairs(w[:1].contiguous(), sets_rows(S, [0]), w[2:].contiguous(), sets_rows(S, [2]), 128)
    e = bs.and_popcount(w[:0].contiguous(), w, 128)
    torch.cuda.synchronize()
    assert e.shape == (0, 3)


@pytest.mark.parametrize("N", [64, 1024, 4096])
def test_measure_scores_fp32_and_fp64(N, dev):
    """bs_estimate_scores: the FP32 matrix of each measure is bit-equal to the
    oracle's FP32 score of every pair (the value bs_topk ranks by), empty and
    full rows included; the FP64 matrix is bs_estimate's plane. 150 x 211
    pairs, popcounts passed for A and computed for B."""
    import torch
    from paper_1910_04658_amd import binding as bs
    c = datagen.saturation_rows(211, N, 61 + N, p_empty=0.05, p_full=0.05, p_near=0.05)
    pi = datagen.identity_map(N)
    w, pop = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    S = oracle.sketch_sets(c.indptr, c.indices, N, pi, N)
    a = np.arange(0, 211, 7).tolist() + list(range(60, 180))
    a = sorted(set(a))[:150]
    A = w[a].contiguous()
    X = oracle.intersections(sets_rows(S, a), S)
    xa, xb = S.length[a], S.length
    planes = bs.estimate(A, w, N)
    for m, key in enumerate(["ip", "ham", "js", "cos"]):
        f32 = bs.estimate_scores(A, w, N, key, torch.float32, popA=pop[a].contiguous())
        f64 = bs.estimate_scores(A, w, N, key, torch.float64)
        torch.cuda.synchronize()
        assert torch.equal(f64, planes[key]), key
        want = np.array([[oracle.score_f32(xa[i], xb[j], X[i, j], N, m) for j in range(len(xb))]
                         for i in range(len(a))], np.float32)
        got = f32.cpu().numpy()
        bad = np.nonzero(got.view(np.uint32) != want.view(np.uint32))
        assert len(bad[0]) == 0, (key, bad[0][:3], bad[1][:3], got[bad][:3], want[bad][:3])
