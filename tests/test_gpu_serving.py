"""The serving loop on the GPU: every request's top-k is the same alone and in
the mix of concurrently batched requests, and equals the CPU oracle."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import to_dev, assert_topk_equal

pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_the_mix(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    from paper_1910_04658_amd.serving import GpuExecutor, Request, Server, make_requests
    N, k = 2048, 50
    corpus = datagen.lognormal_corpus(30000, d=200_000, mean=400.0, sd=300.0, seed=51)
    pi = datagen.random_map(corpus.d, N, 52)
    C, popC = bs.sketch(to_dev(corpus.indptr, dev), to_dev(corpus.indices, dev), to_dev(pi, dev), N)
    q, arr = datagen.serving_queries(150, corpus.d, seed=53, lo=10, hi=5000, rate=4000.0)
    reqs = make_requests(q, arr)
    ex = GpuExecutor(C, popC, to_dev(pi, dev), N, k, "cosine", max_batch=32, n_slots=3, max_nnz=32 * 5000)
    stats = Server(ex, n_slots=3, max_batch=32, mem_budget=1 << 40).run(reqs)
    assert stats["requests"] == 150 and stats["max_batch_seen"] >= 2  # requests were batched together
    # each request alone (a batch of one)
    for r in reqs:
        alone = Request(r.rid, r.indices, 0.0)
        ex.submit(0, [alone])
        idx, sc = ex.results(0)
        assert np.array_equal(idx[0], r.idx) and np.array_equal(sc[0], r.score), r.rid
    # and against the oracle's full sort for a sample of requests
    S = oracle.sketch_sets(corpus.indptr, corpus.indices, corpus.d, pi, N)
    pick = list(range(0, 150, 15))
    sub = q.take(pick)
    SQ = oracle.sketch_sets(sub.indptr, sub.indices, sub.d, pi, N)
    oi, osc = oracle.topk(SQ, S, N, oracle.COS, k)
    gi = np.stack([reqs[i].idx for i in pick])
    gs = np.stack([reqs[i].score for i in pick])
    assert_topk_equal(gi, gs, oi, osc)
