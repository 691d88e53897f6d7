"""Scheduling logic of the serving loop on the CPU: a mock executor answers
with the CPU oracle after a simulated service time, so admission by memory,
batching and completion can be checked without a GPU."""
import time

import numpy as np

import datagen
import oracle
from paper_1910_04658_amd.serving import Request, Server


class MockExecutor:
    def __init__(self, corpus_sets, pi, d, N, k, service_s=0.002):
        self.S, self.pi, self.d, self.N, self.k, self.service = corpus_sets, pi, d, N, k, service_s
        self.max_nnz = 1 << 30
        self.jobs = {}
        self.peak_bytes = 0
        self.live_bytes = 0

    def request_bytes(self, indices):
        return 1000 + 4 * len(indices)

    def submit(self, slot, batch):
        rows = [r.indices for r in batch]
        c = datagen.from_rows(rows, self.d)
        Q = oracle.sketch_sets(c.indptr, c.indices, self.d, self.pi, self.N)
        idx, sc = oracle.topk(Q, self.S, self.N, oracle.COS, self.k)
        self.live_bytes += sum(r.nbytes for r in batch)
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        self.jobs[slot] = (time.perf_counter() + self.service, idx, sc, sum(r.nbytes for r in batch))

    def done(self, slot):
        return time.perf_counter() >= self.jobs[slot][0]

    def results(self, slot):
        _, idx, sc, nb = self.jobs.pop(slot)
        self.live_bytes -= nb
        return idx, sc


def _setup(n_req=60, rate=3000.0):
    corpus = datagen.small_corpus(n=600, d=5000, seed=41)
    N = 256
    pi = datagen.random_map(corpus.d, N, 41)
    S = oracle.sketch_sets(corpus.indptr, corpus.indices, corpus.d, pi, N)
    q, arr = datagen.serving_queries(n_req, corpus.d, seed=42, lo=5, hi=300, rate=rate)
    reqs = [Request(i, q.row(i).astype(np.int32), float(arr[i])) for i in range(q.n)]
    return corpus, N, pi, S, q, reqs


def test_every_request_answered_once_with_oracle_result():
    corpus, N, pi, S, q, reqs = _setup()
    ex = MockExecutor(S, pi, corpus.d, N, k=10)
    stats = Server(ex, n_slots=3, max_batch=8, mem_budget=10 ** 9).run(reqs)
    assert stats["requests"] == len(reqs)
    Q = oracle.sketch_sets(q.indptr, q.indices, corpus.d, pi, N)
    idx, sc = oracle.topk(Q, S, N, oracle.COS, 10)
    for r in reqs:
        assert r.t_done >= r.arrival and r.t_start >= r.arrival - 1e-9
        assert np.array_equal(r.idx, idx[r.rid]) and np.array_equal(r.score, sc[r.rid])


def test_memory_budget_is_never_exceeded_and_limits_batches():
    corpus, N, pi, S, q, reqs = _setup(n_req=80, rate=0.0)  # all arrive at once
    ex = MockExecutor(S, pi, corpus.d, N, k=5)
    budget = max(ex.request_bytes(r.indices) for r in reqs) * 3  # about three requests in flight
    stats = Server(ex, n_slots=4, max_batch=16, mem_budget=budget).run(reqs, realtime=False)
    assert ex.peak_bytes <= budget
    assert stats["max_batch_seen"] <= budget // min(ex.request_bytes(r.indices) for r in reqs)
    assert stats["max_batch_seen"] < 16  # the budget, not the batch size, limited admission
    assert all(r.idx is not None for r in reqs)


def test_fifo_admission_order():
    corpus, N, pi, S, q, reqs = _setup(n_req=40, rate=0.0)
    ex = MockExecutor(S, pi, corpus.d, N, k=5, service_s=0.0005)
    Server(ex, n_slots=2, max_batch=4, mem_budget=10 ** 9).run(reqs, realtime=False)
    starts = [r.t_start for r in reqs]
    assert all(a <= b for a, b in zip(starts, starts[1:]))


def test_request_too_large_for_budget_is_rejected():
    corpus, N, pi, S, q, reqs = _setup(n_req=5)
    ex = MockExecutor(S, pi, corpus.d, N, k=5)
    try:
        Server(ex, n_slots=1, max_batch=4, mem_budget=100).run(reqs)
    except ValueError:
        return
    raise AssertionError("expected a ValueError")
