"""bs_topk against the CPU oracle's full sort: identical indices and FP32
scores (both sides rank by the same FP32 evaluation of the estimators)."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import assert_topk_equal, sets_rows, to_dev

pytestmark = pytest.mark.gpu

MEASURES = [oracle.IP, oracle.HAM, oracle.JS, oracle.COS]


def sketch_both(c, N, seed, dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    pi = datagen.random_map(c.d, N, seed)
    w, _ = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    torch.cuda.synchronize()
    return w, oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)


def gpu_topk(Q, C, N, m, k):
    import torch
    from paper_1910_04658_amd import binding as bs
    i, s = bs.topk(Q, C, N, m, k)
    torch.cuda.synchronize()
    return i.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("m", MEASURES)
def test_corpus_inside_the_sample(m, dev):
    """nC <= 4096: the sample pass covers the whole corpus."""
    c = datagen.small_corpus(n=1000, d=10000, seed=21)
    w, S = sketch_both(c, 1024, 5, dev)
    q = np.arange(0, 1000, 7)
    gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, 1024, m, 25)
    oi, osc = oracle.topk(sets_rows(S, q), S, 1024, m, 25)
    assert_topk_equal(gi, gs, oi, osc)


@pytest.mark.parametrize("m", MEASURES)
@pytest.mark.parametrize("N,k", [(256, 1), (256, 100), (1024, 37), (4096, 100)])
def test_scan_path(m, N, k, dev):
    """nC > 4096: sample, filtered scan and selection."""
    c = datagen.lognormal_corpus(20011, d=30000, seed=22)
    w, S = sketch_both(c, N, 6, dev)
    q = np.arange(0, 20011, 401)
    gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, N, m, k)
    oi, osc = oracle.topk(sets_rows(S, q), S, N, m, k)
    assert_topk_equal(gi, gs, oi, osc)


@pytest.mark.parametrize("m", MEASURES)
@pytest.mark.parametrize("N,nq", [(256, 130), (320, 70), (1024, 65), (8192, 20), (8192, 130), (16384, 33)])
def test_scan_path_query_lanes(m, N, nq, dev):
    """Batches above 64 queries (and widths the row-lane scan does not take:
    N = 320 is not a power-of-two word count; N = 8192 and 16384 exceed 128
    words and take the word-split scan) go through the query-lane scans;
    ragged query counts."""
    c = _mid("c20011", lambda: datagen.lognormal_corpus(20011, d=30000, seed=22))
    w, S = sketch_both(c, N, 6, dev)
    q = np.linspace(0, 20010, nq).astype(np.int64)
    gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, N, m, 40)
    sel = np.arange(0, nq, max(1, nq // 12))
    oi, osc = oracle.topk(sets_rows(S, q[sel]), S, N, m, 40)
    assert_topk_equal(gi[sel], gs[sel], oi, osc)


@pytest.mark.parametrize("m", [oracle.JS, oracle.COS])
@pytest.mark.parametrize("N,nq", [(256, 70), (512, 70), (768, 100), (1024, 130), (4096, 65), (8192, 20),
                                  (16384, 33)])
def test_vector_and_matrix_scans_agree(m, N, nq, dev):
    """Widths of whole 256-bit chunks scan on the matrix cores (FP4 products
    of the sketch bits); with that switched off they take the vector-ALU
    scans (query lanes, or word-split for N >= 8192). Both give the oracle's
    result on sampled queries and identical results on all of them."""
    from paper_1910_04658_amd import binding as bs
    c = _mid("c20011", lambda: datagen.lognormal_corpus(20011, d=30000, seed=22))
    w, S = sketch_both(c, N, 6, dev)
    q = np.linspace(0, 20010, nq).astype(np.int64)
    Q = w[q.tolist()].contiguous()
    gi, gs = gpu_topk(Q, w, N, m, 40)
    try:
        bs.debug_set_topk_mma(False)
        vi, vs = gpu_topk(Q, w, N, m, 40)
    finally:
        bs.debug_set_topk_mma(True)
    sel = np.arange(0, nq, max(1, nq // 8))
    oi, osc = oracle.topk(sets_rows(S, q[sel]), S, N, m, 40)
    assert_topk_equal(gi[sel], gs[sel], oi, osc)
    np.testing.assert_array_equal(gi, vi)
    np.testing.assert_array_equal(gs, vs)


@pytest.mark.parametrize("m", [oracle.JS, oracle.HAM])
@pytest.mark.parametrize("nq", [20, 80])
def test_overflow_fallback_path(m, nq, dev):
    """No candidate slots outside the sample sends every query with a scan
    survivor to the whole-corpus fallback, and one slot sends some; the result
    must not change."""
    from paper_1910_04658_amd import binding as bs
    c = datagen.lognormal_corpus(9000, d=20000, seed=23)
    w, S = sketch_both(c, 512, 7, dev)
    q = np.linspace(0, 8999, nq).astype(np.int64)
    oi, osc = oracle.topk(sets_rows(S, q), S, 512, m, 50)
    for cap in (0, 1):
        try:
            bs.debug_set_topk_limits(slab_capacity=cap)
            gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, 512, m, 50)
        finally:
            bs.debug_set_topk_limits()
        assert_topk_equal(gi, gs, oi, osc)


@pytest.mark.parametrize("m", [oracle.JS, oracle.COS])
@pytest.mark.parametrize("nq", [9, 70])
def test_failed_tau_check_falls_back(m, nq, dev):
    """The filter threshold is the sample's kt-th best score with kt < k; the
    select checks that at least k candidates reach it. Forcing kt down to 1
    or 5 makes the check fail for most queries, which then go to the
    whole-corpus fallback; the result must not change (both scan modes)."""
    from paper_1910_04658_amd import binding as bs
    c = _mid("c30k", lambda: datagen.lognormal_corpus(30000, d=40000, seed=27))
    w, S = sketch_both(c, 512, 11, dev)
    q = np.linspace(0, 29999, nq).astype(np.int64)
    sel = np.arange(0, nq, max(1, nq // 9))
    oi, osc = oracle.topk(sets_rows(S, q[sel]), S, 512, m, 40)
    for rank in (1, 5, -1):
        try:
            bs.debug_set_topk_tau_rank(rank)
            gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, 512, m, 40)
        finally:
            bs.debug_set_topk_tau_rank()
        assert_topk_equal(gi[sel], gs[sel], oi, osc)


@pytest.mark.parametrize("N", [256, 1024])
@pytest.mark.parametrize("lds_keys", [None, 0, 1024])
@pytest.mark.parametrize("nq", [9, 70])
def test_large_candidate_sets_compact_in_place(N, lds_keys, nq, dev):
    """Candidate sets above the LDS buffer are compacted and selected in
    place in global memory. k = 1000 over 60k rows gives ~15k candidates per
    query; the LDS limit is also forced down to send every query (0) or
    most (1024) through the in-place path, for every scan mode (9 queries:
    row lanes; 70: query lanes at N = 256, the matrix cores at N = 1024,
    with many survivors per slab)."""
    from paper_1910_04658_amd import binding as bs
    c = _mid("c60k", lambda: datagen.lognormal_corpus(60000, d=50000, seed=26))
    w, S = sketch_both(c, N, 10, dev)
    q = np.linspace(0, 59999, nq).astype(np.int64)
    sel = np.arange(0, nq, max(1, nq // 9))
    oi, osc = oracle.topk(sets_rows(S, q[sel]), S, N, oracle.JS, 1000)
    try:
        if lds_keys is not None:
            bs.debug_set_topk_limits(lds_keys=lds_keys)
        gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, N, oracle.JS, 1000)
    finally:
        bs.debug_set_topk_limits()
    assert_topk_equal(gi[sel], gs[sel], oi, osc)


@pytest.mark.parametrize("mma", [True, False])
def test_fallback_at_max_k_and_width(mma, dev):
    """No candidate slots outside the sample sends every query with a scan
    survivor to the whole-corpus fallback, here at the largest k (1,024) and
    width (N = 65,536), where the fallback's LDS (the selected keys, a buffer
    of k + 512 keys and the query's 1,024 words) is largest and the buffer is
    cut back to its k best many times; 70 queries, so that the matrix-core
    scan applies (or the vector scan, switched). The result must equal the
    oracle's."""
    from paper_1910_04658_amd import binding as bs
    N = 65536
    c = datagen.lognormal_corpus(3000, d=200_000, mean=400.0, sd=300.0, seed=31)
    w, S = sketch_both(c, N, 12, dev)
    q = np.linspace(0, 2999, 70).astype(np.int64)
    try:
        bs.debug_set_topk_mma(mma)
        bs.debug_set_topk_limits(slab_capacity=0)
        gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, N, oracle.JS, 1024)
    finally:
        bs.debug_set_topk_limits()
        bs.debug_set_topk_mma(True)
    sel = np.arange(0, 70, 10)
    oi, osc = oracle.topk(sets_rows(S, q[sel]), S, N, oracle.JS, 1024)
    assert_topk_equal(gi[sel], gs[sel], oi, osc)


def test_exact_ties_break_by_index(dev):
    """Many identical corpus rows: equal scores, ordered by smaller index."""
    base = datagen.small_corpus(n=50, d=4000, seed=24)
    rows = [base.row(r % 50).tolist() for r in range(6000)]
    c = datagen.from_rows(rows, base.d)
    w, S = sketch_both(c, 256, 8, dev)
    q = np.arange(0, 50, 5)
    for m in MEASURES:
        gi, gs = gpu_topk(w[q.tolist()].contiguous(), w, 256, m, 200)
        oi, osc = oracle.topk(sets_rows(S, q), S, 256, m, 200)
        assert_topk_equal(gi, gs, oi, osc)


def test_k_equals_corpus_size_and_max_k(dev):
    c = datagen.small_corpus(n=1500, d=6000, seed=25)
    w, S = sketch_both(c, 128, 9, dev)
    q = [0, 1, 2]
    gi, gs = gpu_topk(w[q].contiguous(), w[:300].contiguous(), 128, oracle.JS, 300)
    oi, osc = oracle.topk(sets_rows(S, q), sets_rows(S, np.arange(300)), 128, oracle.JS, 300)
    assert_topk_equal(gi, gs, oi, osc)
    gi, gs = gpu_topk(w[q].contiguous(), w, 128, oracle.COS, 1024)
    oi, osc = oracle.topk(sets_rows(S, q), S, 128, oracle.COS, 1024)
    assert_topk_equal(gi, gs, oi, osc)


@pytest.mark.parametrize("N", [256, 1024, 4096])
def test_full_size_query_vs_corpus(N, dev):
    """1,000 queries against 100,000 corpus rows (d = 100,000, log-normal
    lengths), top-100 Jaccard: every query against the oracle's full sort."""
    import torch
    from paper_1910_04658_amd import binding as bs
    corpus = _big("corpus", lambda: datagen.lognormal_corpus(100_000))
    queries = _big("queries", lambda: datagen.lognormal_corpus(1000, seed=datagen.SEED_QUERIES))
    pi = datagen.random_map(corpus.d, N, datagen.SEED_PI + N)
    C, _ = bs.sketch(to_dev(corpus.indptr, dev), to_dev(corpus.indices, dev), to_dev(pi, dev), N)
    Q, _ = bs.sketch(to_dev(queries.indptr, dev), to_dev(queries.indices, dev), to_dev(pi, dev), N)
    idx, sc = bs.topk(Q, C, N, "js", 100)
    torch.cuda.synchronize()
    SC = oracle.sketch_sets(corpus.indptr, corpus.indices, corpus.d, pi, N)
    SQ = oracle.sketch_sets(queries.indptr, queries.indices, queries.d, pi, N)
    oi, osc = oracle.topk(SQ, SC, N, oracle.JS, 100)
    assert_topk_equal(idx.cpu().numpy(), sc.cpu().numpy(), oi, osc)


@pytest.mark.parametrize("N,nq", [(256, 70), (1024, 9), (1024, 70), (4096, 130), (16384, 70), (32768, 70),
                                  (65536, 9), (65536, 70)])
def test_empty_and_saturated_rows(N, nq, dev):
    """Empty rows (Jaccard and cosine 0/0, scored 0), full rows (x = N: the
    saturation clamp) and rows missing a few coordinates, in the corpus and
    the queries, sketched through the identity map so each row is its own
    sketch. The last query is full, so in a ragged batch the query slots past
    the batch (which hold the last query's words) meet full corpus rows with
    x_ab = N; they must store nothing. Every scan that applies runs: the
    matrix cores (N a multiple of 256, more than 64 queries or N > 4096) and
    the vector ALU with them switched off (query lanes, word split, any width;
    row lanes for 9 queries up to N = 4096). All queries and all four
    measures against the oracle's full sort."""
    from paper_1910_04658_amd import binding as bs
    big = N > 8192
    c = datagen.saturation_rows(6000, N, 31, p_full=0.01 if big else 0.03, p_near=0.01 if big else 0.06)
    qs = datagen.saturation_rows(nq, N, 32, p_empty=0.06, p_full=0.06, p_near=0.06, last_full=True)
    pi = datagen.identity_map(N)
    C, _ = bs.sketch(to_dev(c.indptr, dev), to_dev(c.indices, dev), to_dev(pi, dev), N)
    Q, _ = bs.sketch(to_dev(qs.indptr, dev), to_dev(qs.indices, dev), to_dev(pi, dev), N)
    SC = oracle.sketch_sets(c.indptr, c.indices, N, pi, N)
    SQ = oracle.sketch_sets(qs.indptr, qs.indices, N, pi, N)
    assert SQ.length[-1] == N and (SC.length == N).any() and (SC.length == 0).any()
    modes = [True, False] if N % 256 == 0 and (nq > 64 or N > 4096) else [True]
    for m in MEASURES:
        oi, osc = oracle.topk(SQ, SC, N, m, 50)
        for mma in modes:
            try:
                bs.debug_set_topk_mma(mma)
                gi, gs = gpu_topk(Q, C, N, m, 50)
            finally:
                bs.debug_set_topk_mma(True)
            assert_topk_equal(gi, gs, oi, osc)


def _mid(key, fn):
    from conftest import shared_input
    return shared_input(key, fn)


def _big(key, fn):
    from conftest import shared_input
    return shared_input({"corpus": "corpus100k", "queries": "queries1k"}[key], fn)
