"""Continuous-batching query server over a device-resident sketched corpus.

Requests (one sparse binary query vector each) arrive over time. The server
keeps up to `n_slots` batches in flight, one per HIP stream, so their work
overlaps on the device. Whenever a slot is free it admits the pending
requests in arrival order, as many as fit both the batch size and the memory
budget (bytes of query data plus each query's share of the top-k workspace),
sketches them (bs_sketch) and ranks them against the corpus (bs_topk). A slot's
requests complete when its stream has finished; latency is measured from
arrival to the moment the server observes completion.

Each query's result depends only on that query and the corpus (bs_topk
selects per query), so a request gets the same answer alone or in any mix.

The scheduler talks to an executor with three calls (submit, done, results):
GpuExecutor drives the library; tests can drive the same scheduler with a CPU
executor that has the same interface.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import binding as bs


@dataclasses.dataclass
class Request:
    rid: int
    indices: np.ndarray   # int32 set indices of the query vector
    arrival: float        # seconds since the start of the run
    nbytes: int = 0       # memory charged to admission
    t_start: float = -1.0
    t_done: float = -1.0
    idx: np.ndarray | None = None
    score: np.ndarray | None = None
    slot: int = -1


class GpuExecutor:
    """Sketch + top-k of a batch of queries on one stream per slot; every
    buffer is allocated up front for batches of up to `max_batch` queries."""

    def __init__(self, corpus: torch.Tensor, corpus_pop: torch.Tensor, pi: torch.Tensor, N: int, k: int,
                 measure: str, max_batch: int, n_slots: int, max_nnz: int):
        self.dev = corpus.device
        self.C, self.popC, self.pi, self.N, self.k, self.measure = corpus, corpus_pop, pi, N, k, measure
        self.nC = corpus.shape[0]
        self.max_batch, self.n_slots, self.max_nnz = max_batch, n_slots, max_nnz
        W = N // 64
        ws_k = bs.topk_workspace_size(max_batch, self.nC, N, k)
        ws_s = bs.sketch_workspace_size(pi.numel(), N)
        self.slots = []
        for _ in range(n_slots):
            st = torch.cuda.Stream(device=self.dev)
            self.slots.append({
                "stream": st,
                "event": torch.cuda.Event(),
                "indptr": torch.empty(max_batch + 1, dtype=torch.int32, device=self.dev),
                "indices": torch.empty(max(max_nnz, 1), dtype=torch.int32, device=self.dev),
                "h_indptr": torch.empty(max_batch + 1, dtype=torch.int32, pin_memory=True),
                "h_indices": torch.empty(max(max_nnz, 1), dtype=torch.int32, pin_memory=True),
                "Q": torch.empty((max_batch, W), dtype=torch.int64, device=self.dev),
                "popQ": torch.empty(max_batch, dtype=torch.int32, device=self.dev),
                "idx": torch.empty((max_batch, k), dtype=torch.int32, device=self.dev),
                "score": torch.empty((max_batch, k), dtype=torch.float32, device=self.dev),
                "h_idx": torch.empty((max_batch, k), dtype=torch.int32, pin_memory=True),
                "h_score": torch.empty((max_batch, k), dtype=torch.float32, pin_memory=True),
                "ws_topk": bs._workspace(ws_k, self.dev),
                "ws_sketch": bs._workspace(ws_s, self.dev),
                "n": 0,
            })
        torch.cuda.synchronize(self.dev)
        self.per_query_ws = max(0, bs.topk_workspace_size(2, self.nC, N, k) - bs.topk_workspace_size(1, self.nC, N, k))

    def request_bytes(self, indices: np.ndarray) -> int:
        """Device memory a request occupies while in flight: its indices, its
        sketch and popcount, its results and its share of the top-k workspace."""
        return 4 * (len(indices) + 1) + self.N // 8 + 4 + 8 * self.k + self.per_query_ws

    def submit(self, slot: int, batch: list):
        s = self.slots[slot]
        n = len(batch)
        lens = np.fromiter((len(r.indices) for r in batch), dtype=np.int64, count=n)
        nnz = int(lens.sum())
        if n > self.max_batch or nnz > self.max_nnz:
            raise ValueError("batch exceeds the executor's preallocated buffers")
        hp = s["h_indptr"].numpy()
        hp[0] = 0
        np.cumsum(lens, out=hp[1:n + 1])
        hi = s["h_indices"].numpy()
        if nnz:
            hi[:nnz] = np.concatenate([r.indices for r in batch])
        with torch.cuda.stream(s["stream"]):
            s["indptr"][:n + 1].copy_(s["h_indptr"][:n + 1], non_blocking=True)
            s["indices"][:max(nnz, 1)].copy_(s["h_indices"][:max(nnz, 1)], non_blocking=True)
            Q, popQ = s["Q"][:n], s["popQ"][:n]
            bs.sketch(s["indptr"][:n + 1], s["indices"][:nnz], self.pi, self.N, out=Q, popcounts=popQ,
                      workspace=s["ws_sketch"])
            bs.topk(Q, self.C, self.N, self.measure, self.k, workspace=s["ws_topk"], out_idx=s["idx"][:n],
                    out_score=s["score"][:n], popQ=popQ, popC=self.popC)
            s["h_idx"][:n].copy_(s["idx"][:n], non_blocking=True)
            s["h_score"][:n].copy_(s["score"][:n], non_blocking=True)
            s["event"].record(s["stream"])
        s["n"] = n

    def done(self, slot: int) -> bool:
        return self.slots[slot]["event"].query()

    def results(self, slot: int):
        s = self.slots[slot]
        s["event"].synchronize()
        n = s["n"]
        return s["h_idx"][:n].numpy().copy(), s["h_score"][:n].numpy().copy()


class Server:
    """Continuous batching with memory-based admission (see the module notes)."""

    def __init__(self, executor, n_slots: int, max_batch: int, mem_budget: int, max_nnz: int | None = None):
        self.ex, self.n_slots, self.max_batch, self.budget = executor, n_slots, max_batch, mem_budget
        self.max_nnz = max_nnz if max_nnz is not None else getattr(executor, "max_nnz", 1 << 62)

    def run(self, requests: list, realtime: bool = True, clock=time.perf_counter):
        """Serve `requests` (sorted by arrival); returns statistics. With
        realtime=False every request is available at time 0 (offline)."""
        for r in requests:
            r.nbytes = self.ex.request_bytes(r.indices)
            if r.nbytes > self.budget or len(r.indices) > self.max_nnz:
                raise ValueError("request %d can never be admitted under the memory budget" % r.rid)
        pending = collections.deque()
        in_flight = {}           # slot -> list of requests
        used = 0                 # bytes of admitted, unfinished requests
        free = list(range(self.n_slots))
        i, done, n = 0, 0, len(requests)
        batches = []
        t0 = clock()
        while done < n:
            now = clock() - t0
            while i < n and (not realtime or requests[i].arrival <= now):
                pending.append(requests[i])
                i += 1
            progressed = False
            for slot in list(in_flight):
                if self.ex.done(slot):
                    idx, score = self.ex.results(slot)
                    t = clock() - t0
                    for j, r in enumerate(in_flight[slot]):
                        r.idx, r.score, r.t_done = idx[j], score[j], t
                        used -= r.nbytes
                    done += len(in_flight[slot])
                    del in_flight[slot]
                    free.append(slot)
                    progressed = True
            while free and pending:
                batch, b_bytes, b_nnz = [], 0, 0
                while pending and len(batch) < self.max_batch:
                    r = pending[0]
                    if used + b_bytes + r.nbytes > self.budget or b_nnz + len(r.indices) > self.max_nnz:
                        break
                    batch.append(pending.popleft())
                    b_bytes += r.nbytes
                    b_nnz += len(r.indices)
                if not batch:
                    break  # waits for memory to be released
                slot = free.pop()
                t = clock() - t0
                for r in batch:
                    r.t_start, r.slot = t, slot
                self.ex.submit(slot, batch)
                in_flight[slot] = batch
                used += b_bytes
                batches.append(len(batch))
                progressed = True
            if not progressed:
                time.sleep(20e-6)
        wall = clock() - t0
        lat = np.array([r.t_done - (r.arrival if realtime else 0.0) for r in requests])
        return {"requests": n, "wall_s": wall, "throughput_qps": n / wall,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_batch": float(np.mean(batches)) if batches else 0.0, "batches": len(batches),
                "max_batch_seen": int(max(batches)) if batches else 0}


def make_requests(q_csr, arrivals) -> list:
    return [Request(rid=i, indices=np.ascontiguousarray(q_csr.row(i), dtype=np.int32), arrival=float(arrivals[i]))
            for i in range(q_csr.n)]
