#!/usr/bin/env python3
"""BinSketch hot-path benchmark on one MI355X.

One step = the whole hot path over one batch of synthetic input:
  1. sketch the corpus: 100,000 binary vectors, d = 100,000, row lengths
     round(log-normal) with mean 230 and sd 150, Zipf(1.1) feature popularity;
  2. sketch the queries: 1,000 vectors from the same generator, another seed;
  3. score every query against every corpus row by the Jaccard estimator and
     keep the top 100 per query (FP32 scores).
at sketch width N = 1024 (also reported: N = 256 and N = 4096).

Inputs are resident in device memory before timing starts. The timed
region is exactly `--steps` steps between two device synchronisations
(`--graph`: replays of the step recorded into a HIP graph). Per-kernel launch
durations come from a separate eager pass, from HIP events that the library
records on the launching stream while timing is enabled.

Printed: one JSON line (see the keys below). `value` is pair estimates per
second of the whole step (sketching included). `vector_scan` repeats the step
at the metric's width with the pair counts on the vector ALU (the matrix
cores switched off) and gives that scan's int32 VALU roofline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# int32 VALU: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_FP4_TFLOPS = 10100.0  # dense FP4 matrix-core peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "topk_scan": ["paper_1910_04658_amd/csrc/topk.hip", "paper_1910_04658_amd/csrc/bs_common.h"],
    "sketch_csr": ["paper_1910_04658_amd/csrc/sketch.hip", "paper_1910_04658_amd/csrc/bs_common.h"],
}


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/traffic.json),
    or None when no record exists or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))[kernel][workload]
    except (KeyError, ValueError):
        return None
    if rec.get("src_sha") != src_digest(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("hbm_bytes_per_launch")


def ingest_counters(fetch_dir, write_dir, copy_bytes, N):
    """HBM bytes per launch of the dominant kernels from rocprofv3 counter runs.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by the factor that
    makes the same counter read exactly the known size of a plain copy kernel
    (the `--copy-bytes` run profiled in the same directory)."""
    import csv
    import glob

    copy_bytes = int(copy_bytes)

    def per_kernel(d, counter):
        out = {}
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r["Counter_Name"] != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return out

    res = {}
    seen = {}  # short name -> the full kernel names counted under it
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        k = per_kernel(d, counter)
        copy = [v for name, vals in k.items() if "copy" in name.lower() or "elementwise" in name.lower()
                for v in vals if v > copy_bytes * 0.25]
        if not copy:
            raise SystemExit("no copy-kernel dispatch found in %s" % d)
        factor = copy_bytes / max(copy)
        for name, vals in k.items():
            for short in KERNEL_SOURCES:
                if short + "_" in name or short + "_lds" in name or name.split("(")[0].endswith(short + "_kernel"):
                    seen.setdefault(short, set()).add(name)
                    res.setdefault(short, {})[counter] = (sum(vals) / len(vals), factor, len(vals))
    for short, names in seen.items():
        if len(names) > 1:  # one figure per kernel: a run that mixes variants cannot be ingested
            raise SystemExit("%s: %d kernel variants in the counter run (%s); profile one variant, e.g. with "
                             "--no-vector-scan" % (short, len(names), "; ".join(sorted(n[:80] for n in names))))
    out = {}
    for short, c in res.items():
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fb, ff, nf = c["FETCH_SIZE"]
        wb, wf, nw = c["WRITE_SIZE"]
        out[short] = {"N%d" % N: {"src_sha": src_digest(KERNEL_SOURCES[short]),
                                  "hbm_bytes_per_launch": fb * ff + wb * wf,
                                  "fetch_bytes_raw": fb, "fetch_factor": ff, "write_bytes_raw": wb,
                                  "write_factor": wf, "dispatches": [nf, nw]}}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    old = json.load(open(path)) if os.path.exists(path) else {}
    for short, v in out.items():
        old.setdefault(short, {}).update(v)
    with open(path, "w") as f:
        json.dump(old, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1))


def make_inputs(N_list, dev):
    import torch

    import datagen
    t = time.time()
    corpus = datagen.lognormal_corpus(100_000, d=100_000, mean=230.0, sd=150.0, seed=datagen.SEED_CORPUS)
    queries = datagen.lognormal_corpus(1000, d=100_000, mean=230.0, sd=150.0, seed=datagen.SEED_QUERIES)
    log("inputs generated in %.1fs: corpus nnz %d (mean %.1f), queries nnz %d" % (
        time.time() - t, corpus.nnz, corpus.nnz / corpus.n, queries.nnz))
    pis = {N: datagen.random_map(corpus.d, N, datagen.SEED_PI + N) for N in N_list}
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    dev_in = {"c_indptr": to(corpus.indptr), "c_indices": to(corpus.indices),
              "q_indptr": to(queries.indptr), "q_indices": to(queries.indices),
              "pi": {N: to(p) for N, p in pis.items()}}
    return corpus, queries, pis, dev_in


class Step:
    """Preallocated outputs and workspace for one width N."""

    def __init__(self, dev_in, N, k, nC, nQ, dev):
        import torch

        from paper_1910_04658_amd import binding as bs
        self.bs = bs
        self.N, self.k = N, k
        W = N // 64
        self.d = dev_in
        self.pi = dev_in["pi"][N]
        self.C = torch.empty((nC, W), dtype=torch.int64, device=dev)
        self.Q = torch.empty((nQ, W), dtype=torch.int64, device=dev)
        self.popC = torch.empty(nC, dtype=torch.int32, device=dev)
        self.popQ = torch.empty(nQ, dtype=torch.int32, device=dev)
        self.idx = torch.empty((nQ, k), dtype=torch.int32, device=dev)
        self.score = torch.empty((nQ, k), dtype=torch.float32, device=dev)
        self.ws = bs._workspace(bs.topk_workspace_size(nQ, nC, N, k), dev)
        # the map is fixed per (d, N): bit-packed once, before timing (like
        # drawing it, this is not part of a step)
        self.packed = bs.prepare_map(self.pi, N)

    def __call__(self):
        bs, d = self.bs, self.d
        # corpus and queries share the map: one sketch launch
        bs.sketch_parts([(d["c_indptr"], d["c_indices"]), (d["q_indptr"], d["q_indices"])], self.pi, self.N,
                        outs=[self.C, self.Q], popcounts=[self.popC, self.popQ], prepared=self.packed)
        bs.topk(self.Q, self.C, self.N, "js", self.k, workspace=self.ws, out_idx=self.idx,
                out_score=self.score, popQ=self.popQ, popC=self.popC)


def timed(step, steps, warmup, graph=False):
    """ms per step and per-kernel mean launch times.

    Eager launches by default; graph=True records the step's launches (two
    sketches and the top-k stages) once into a HIP graph and times replays.
    Kernel times come from a separate eager pass with the library's HIP-event
    timing on (events inside the timed region would add to it)."""
    import torch
    bs = step.bs
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    run = step
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel timing, eager
    bs.timing_collect()
    bs.timing_reset()
    bs.timing_enable(True)
    n_timed = min(steps, 20)
    for _ in range(n_timed):
        step()
    torch.cuda.synchronize()
    bs.timing_enable(False)
    bad = bs.timing_collect()
    kt = {}
    for name in ["sketch_pack", "sketch_csr", "topk_prep", "topk_sample", "topk_sample_select", "topk_bound",
                 "topk_scan", "topk_select"]:
        ms, n = bs.timing_get(name)
        if n:
            kt[name] = {"avg_ms": ms / n, "launches": n, "per_step": n / n_timed}
    if bad:
        log("warning: %d kernel timing events could not be read" % bad)
    return (t1 - t0) * 1e3 / steps, kt


def jaccard_mse(step, corpus, queries):
    """Closed-form Jaccard estimates vs exact Jaccard on (a) every pair of the
    1,000 queries with the first 2,000 corpus rows and (b) the returned top-100
    pairs. Exact values by sparse products on the host."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    bs = step.bs

    def mat(c, rows=None):
        m = sp.csr_matrix((np.ones(c.nnz, np.float64), c.indices, c.indptr), shape=(c.n, c.d))
        return m if rows is None else m[rows]

    Qm = mat(queries)
    Cm = mat(corpus, np.arange(2000))
    inter = (Qm @ Cm.T).toarray()
    la = np.asarray(Qm.sum(1)).ravel()[:, None]
    lb = np.asarray(Cm.sum(1)).ravel()[None, :]
    exact = inter / (la + lb - inter)
    est = bs.estimate(step.Q, step.C[:2000].contiguous(), step.N, measures=("js",))["js"]
    torch.cuda.synchronize()
    mse_random = float(np.mean((est.cpu().numpy() - exact) ** 2))
    idx = step.idx.cpu().numpy()
    sc = step.score.cpu().numpy().astype(np.float64)
    Cfull = mat(corpus)
    errs = []
    for q in range(0, idx.shape[0], 10):
        sub = Cfull[idx[q]]
        it = np.asarray((Qm[q] @ sub.T).todense()).ravel()
        lbq = np.asarray(sub.sum(1)).ravel()
        ex = it / (la[q, 0] + lbq - it)
        errs.append((sc[q] - ex) ** 2)
    mse_top = float(np.mean(np.concatenate(errs)))
    mean_js_top = float(np.mean(sc[::10]))
    return {"random_pairs": mse_random, "random_pairs_n": int(exact.size),
            "top100_pairs": mse_top, "top100_mean_estimate": mean_js_top}


def dense_eval(dev, reps=50):
    """All-pairs estimates of the small corpus (1,000 vectors, d = 10,000,
    Zipf(1.1) lengths in [5, 500], N = 1024): sketch, then all 1,000 x 1,000
    IP / Hamming / Jaccard / cosine estimates in FP64 (Algorithms 1-4), 32 MB
    of output. The estimate kernel is bound by its HBM writes."""
    import torch

    import datagen
    from paper_1910_04658_amd import binding as bs
    N = 1024
    c = datagen.small_corpus()
    pi = datagen.random_map(c.d, N, datagen.SEED_PI)
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    indptr, indices, pi_d = to(c.indptr), to(c.indices), to(pi)
    n = c.n
    W = torch.empty((n, N // 64), dtype=torch.int64, device=dev)
    pop = torch.empty(n, dtype=torch.int32, device=dev)
    outs = {k: torch.empty((n, n), dtype=torch.float64, device=dev) for k in ("ip", "ham", "js", "cos")}
    sws = bs._workspace(bs.sketch_workspace_size(c.d, N), dev)
    L = bs.load()
    ews = bs._workspace(L.bs_estimate_workspace_size(n, n, N), dev)

    def step():
        bs.sketch(indptr, indices, pi_d, N, out=W, popcounts=pop, workspace=sws)
        st = L.bs_estimate(bs._ptr(W), bs._ptr(pop), n, bs._ptr(W), bs._ptr(pop), n, N, bs._ptr(outs["ip"]),
                           bs._ptr(outs["ham"]), bs._ptr(outs["js"]), bs._ptr(outs["cos"]), bs._ptr(ews),
                           ews.numel(), bs._stream())
        bs._check(st, "bs_estimate")
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    bs.timing_collect()
    bs.timing_reset()
    bs.timing_enable(True)
    for _ in range(10):
        step()
    torch.cuda.synchronize()
    bs.timing_enable(False)
    bs.timing_collect()
    est_ms, cnt = bs.timing_get("pair_estimate")
    est_ms /= max(cnt, 1)
    # algorithmic bytes of the estimate launch: 4 planes of n*n doubles
    # written, both sketch matrices and popcounts read once
    by = 4 * n * n * 8 + 2 * n * (N // 8) + 2 * n * 4
    ach = by / (est_ms * 1e-3) / 1e9
    return {"workload": "all-pairs estimates, 1,000 x 1,000 (diagonal included), N = 1024, FP64, 4 measures",
            "rows": n, "nnz": int(c.nnz), "ms_per_step": ms, "pair_estimates_per_s": n * n / (ms * 1e-3),
            "estimate_kernel_ms": est_ms,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": ach / PEAK_HBM_GBS, "bytes_per_launch": by, "kernel": "pair_estimate"}}


def ranking_eval(dev, max_queries=500, widths=(256, 1024, 4096)):
    """Threshold retrieval (Section 4.2, Experiment 2) on synthetic rows with
    planted near-duplicates, split 90/10 into corpus and queries: for every
    query the corpus rows whose similarity reaches each of the paper's
    thresholds, from bs_estimate on the sketches against the exact
    similarities (sparse products on the host); accuracy, precision, recall
    and F1 pooled over (query, row) pairs, per sketch width."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    import datagen
    from paper_1910_04658_amd import binding as bs
    from paper_1910_04658_amd import ranking
    corpus, queries = datagen.ranking_split()
    queries = queries.take(np.arange(min(max_queries, queries.n)))

    def mat(c):
        return sp.csr_matrix((np.ones(c.nnz, np.float64), c.indices, c.indptr), shape=(c.n, c.d))

    Qm, Cm = mat(queries), mat(corpus)
    inter = (Qm @ Cm.T).toarray()
    la = np.asarray(Qm.sum(1)).ravel()[:, None]
    lb = np.asarray(Cm.sum(1)).ravel()[None, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        exact = {"ip": inter,
                 "js": np.where(la + lb - inter > 0, inter / (la + lb - inter), 0.0),
                 "cos": np.where(la * lb > 0, inter / np.sqrt(la * lb), 0.0)}
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    parts = [(to(corpus.indptr), to(corpus.indices)), (to(queries.indptr), to(queries.indices))]
    out = {"corpus_rows": corpus.n, "queries": queries.n, "pairs": int(inter.size), "thresholds": list(ranking.THRESHOLDS),
           "ip_thresholds": "fractions of the largest exact inner product", "widths": {}}
    for N in widths:
        pi = to(datagen.random_map(corpus.d, N, datagen.SEED_PI + 11 + N))
        (C, pC), (Q, pQ) = bs.sketch_parts(parts, pi, N)
        est = bs.estimate(Q, C, N, measures=("ip", "js", "cos"), popA=pQ, popB=pC)
        torch.cuda.synchronize()
        res = {}
        for m in ("js", "cos", "ip"):
            e = est[m].cpu().numpy()
            th = ranking.ip_thresholds(exact["ip"]) if m == "ip" else ranking.THRESHOLDS
            met = ranking.threshold_metrics(e, exact[m], th)
            res[m] = [[round(t, 4), round(v["accuracy"], 4), round(v["precision"], 4), round(v["recall"], 4),
                       round(v["f1"], 4), v["truth"], v["found"]] for t, v in met.items()]
        out["widths"][str(N)] = res
        del est
    out["columns"] = ["threshold", "accuracy", "precision", "recall", "f1", "truth_pairs", "found_pairs"]
    return out


def learned_eval(dev, n_train_groups=20000, n_test_groups=2000, group=32, N=256, steps=(600, 1500, 3000, 6000),
                 batch=65536):
    """Learned estimator vs closed form: train on ~10M near-duplicate pairs of
    the benchmark distribution sketched at N = 256, test on ~1M held-out pairs.
    One network per training length (cosine schedule over its own length), so
    the held-out MSE against the step count shows where training converges;
    the longest run is also scored per saturation bucket of x_u / N
    (x_u = |a_s OR b_s|), next to the closed form and to the empirical mean
    label of each exact count triple seen in training (a lookup-table
    predictor, the reference for what the three counts allow)."""
    import numpy as np
    import torch

    import datagen
    from paper_1910_04658_amd import binding as bs
    from paper_1910_04658_amd import learned
    t = time.time()
    tr = datagen.variant_groups(n_train_groups, group, seed=5005)
    te = datagen.variant_groups(n_test_groups, group, seed=6006)
    pi = datagen.random_map(tr.csr.d, N, datagen.SEED_PI + 7)
    t_gen = time.time() - t
    dtr = learned.sketch_pairs(tr, pi, N, dev)
    dte = learned.sketch_pairs(te, pi, N, dev)
    del tr, te
    base = learned.closed_form(dte)
    curve = []
    model = None
    for st in steps:
        model = learned.Model(learned.init_master(0, dev))
        torch.cuda.synchronize()
        t = time.time()
        model.train(dtr, steps=st, batch=batch, lr=3e-3, seed=0)
        torch.cuda.synchronize()
        curve.append({"steps": st, "train_seconds": time.time() - t,
                      "mse_learned": learned.mse(model.predict(dte), dte)})
    pred = model.predict(dte)
    out = {"N": N, "train_pairs": len(dtr), "heldout_pairs": len(dte), "batch": batch, "steps": steps[-1],
           "mse_learned": curve[-1]["mse_learned"], "mse_closed_form": learned.mse(base, dte),
           "train_seconds": curve[-1]["train_seconds"], "data_seconds": t_gen, "convergence": curve}

    # per-bucket errors on the held-out pairs
    xa, xb, xab = (v.cpu().numpy().astype(np.int64) for v in (dte.xa, dte.xb, dte.xab))
    lab = dte.label.cpu().numpy().astype(np.float64)
    pl = pred.cpu().numpy().astype(np.float64)
    pc = base.cpu().numpy().astype(np.float64)
    # lookup-table reference: mean training label per exact (x_a, x_b, x_ab)
    txa, txb, txab = (v.cpu().numpy().astype(np.int64) for v in (dtr.xa, dtr.xb, dtr.xab))
    M = N + 1
    tkey = (txa * M + txb) * M + txab
    keys, inv = np.unique(tkey, return_inverse=True)
    tmean = np.bincount(inv, weights=dtr.label.cpu().numpy().astype(np.float64)) / np.bincount(inv)
    hkey = (xa * M + xb) * M + xab
    pos = np.clip(np.searchsorted(keys, hkey), 0, len(keys) - 1)
    seen = keys[pos] == hkey
    plut = np.where(seen, tmean[pos], np.nan)
    xu = (xa + xb - xab) / N
    edges = [0.0, 0.5, 0.75, 0.9, 0.97, 1.0001]
    buckets = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (xu >= lo) & (xu < hi)
        ms = m & seen
        if not m.any():
            continue
        buckets.append({"xu_over_N": [lo, min(hi, 1.0)], "pairs": int(m.sum()),
                        "mse_learned": float(np.mean((pl[m] - lab[m]) ** 2)),
                        "mse_closed_form": float(np.mean((pc[m] - lab[m]) ** 2)),
                        "lookup_coverage": float(ms.sum() / m.sum()),
                        "mse_lookup_on_covered": float(np.mean((plut[ms] - lab[ms]) ** 2)) if ms.any() else None,
                        "mse_learned_on_covered": float(np.mean((pl[ms] - lab[ms]) ** 2)) if ms.any() else None})
    out["by_saturation"] = buckets
    out["lookup_reference"] = {"coverage": float(seen.mean()),
                               "mse_lookup_on_covered": float(np.mean((plut[seen] - lab[seen]) ** 2)),
                               "mse_learned_on_covered": float(np.mean((pl[seen] - lab[seen]) ** 2)),
                               "mse_closed_form_on_covered": float(np.mean((pc[seen] - lab[seen]) ** 2))}
    # inference throughput on the held-out pairs
    ws = bs.mlp_workspace(len(dte), N, dev)
    o = torch.empty(len(dte), dtype=torch.float32, device=dev)
    for _ in range(3):
        bs.mlp_forward(model.w, dte.xa, dte.xb, dte.xab, N, out=o, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(20):
        bs.mlp_forward(model.w, dte.xa, dte.xb, dte.xab, N, out=o, workspace=ws)
    torch.cuda.synchronize()
    out["infer_pairs_per_s"] = 20 * len(dte) / (time.perf_counter() - t)
    return out


def serving_eval(dev, n_corpus=10_000_000, d=1_000_000, N=2048, k=50, n_req=4000, rate=2000.0,
                 n_slots=3, max_batch=64):
    """Continuous-batching server over a device-resident corpus of n_corpus
    vectors (d = 10^6, lognormal lengths mean 400 sd 300, Zipf(1.1) ids),
    sketched at N = 2048; queries of 10-5,000 set bits arrive as a Poisson
    process at `rate` per second and get a top-50 cosine ranking."""
    import torch

    import datagen
    from paper_1910_04658_amd import binding as bs
    from paper_1910_04658_amd.serving import GpuExecutor, Server, make_requests
    t = time.time()
    pi = datagen.random_map(d, N, datagen.SEED_PI + 11)
    pi_d = torch.from_numpy(pi).to(dev)
    C = torch.empty((n_corpus, N // 64), dtype=torch.int64, device=dev)
    popC = torch.empty(n_corpus, dtype=torch.int32, device=dev)
    ws = bs._workspace(bs.sketch_workspace_size(d, N), dev)
    r0 = 0
    nnz = 0
    for indptr, indices in datagen.device_corpus_chunks(n_corpus, d, 400.0, 300.0, seed=7007, device=dev,
                                                         chunk_rows=1 << 18, hi=5000):
        m = indptr.numel() - 1
        bs.sketch(indptr, indices, pi_d, N, out=C[r0:r0 + m], popcounts=popC[r0:r0 + m], workspace=ws)
        r0 += m
        nnz += indices.numel()
    torch.cuda.synchronize()
    t_build = time.time() - t
    q, arr = datagen.serving_queries(n_req, d, seed=8008, lo=10, hi=5000, rate=rate)
    ex = GpuExecutor(C, popC, pi_d, N, k, "cosine", max_batch=max_batch, n_slots=n_slots,
                     max_nnz=max_batch * 5000)
    budget = 16 << 30
    srv = Server(ex, n_slots=n_slots, max_batch=max_batch, mem_budget=budget)
    srv.run(make_requests(q, arr)[:200], realtime=False)  # warm-up
    online = srv.run(make_requests(q, arr), realtime=True)
    offline = srv.run(make_requests(q, arr), realtime=False)
    return {"corpus_rows": n_corpus, "corpus_nnz": nnz, "d": d, "N": N, "k": k, "measure": "cosine",
            "corpus_sketch_GB": C.numel() * 8 / 1e9, "corpus_build_s": t_build,
            "arrival_rate_qps": rate, "requests": n_req, "slots": n_slots, "max_batch": max_batch,
            "mem_budget_GB": budget / 2 ** 30,
            "online": online, "offline_all_at_once": offline}


def batch_eval(dev, n_problems=64, k=100, reps=5, check=4):
    """64 independent problems (sizes 1k-200k rows, d 1e4-1e6, mean row
    weight 20-2,000, N in {128, 512, 2048, 8192}, queries 1% of the rows, at
    least 100; top-100 Jaccard) sketched and ranked by one graph launch after
    autotuning, against the same problems run one after another through
    bs_sketch and bs_topk."""
    import torch

    import datagen
    from paper_1910_04658_amd import binding as bs
    t = time.time()
    specs = datagen.batch_specs(n_problems)
    probs = datagen.device_batch(specs, dev, k=k)
    torch.cuda.synchronize()
    t_gen = time.time() - t
    rows = sum(sp.n + sp.nq for sp in specs)
    pairs = sum(sp.n * sp.nq for sp in specs)
    nnz = sum(p["indices"].numel() + p["q_indices"].numel() for p in probs)
    b = bs.Batch(probs, "js")
    t = time.time()
    b.autotune(reps=2)
    torch.cuda.synchronize()
    t_tune = time.time() - t
    b.run()  # records the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / reps

    def one_by_one():
        outs = []
        for p in probs:
            C, pC = bs.sketch(p["indptr"], p["indices"], p["pi"], p["N"])
            Q, pQ = bs.sketch(p["q_indptr"], p["q_indices"], p["pi"], p["N"])
            ws = bs._workspace(bs.topk_workspace_size(Q.shape[0], C.shape[0], p["N"], p["k"]), dev)
            outs.append((C, ws, bs.topk(Q, C, p["N"], "js", p["k"], popQ=pQ, popC=pC, workspace=ws)))
        return outs
    single = one_by_one()  # warm-up, and the reference results
    torch.cuda.synchronize()
    same = all(torch.equal(b.out[i]["idx"], single[i][2][0]) and torch.equal(b.out[i]["sketches"], single[i][0])
               for i in range(min(check, len(probs))))
    del single
    e0.record()
    for _ in range(2):
        one_by_one()
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / 2
    out = {"problems": n_problems, "rows_sketched": rows, "nnz": nnz, "pair_estimates": pairs,
           "widths": sorted({sp.N for sp in specs}), "k": k, "measure": "jaccard",
           "graph_ms": ms_graph, "graph_nodes": b.graph_nodes(),
           "vectors_per_s": rows / (ms_graph * 1e-3), "pair_estimates_per_s": pairs / (ms_graph * 1e-3),
           "one_by_one_ms": ms_single, "speedup_vs_one_by_one": ms_single / ms_graph,
           "same_as_one_by_one": bool(same), "autotune_s": t_tune, "shapes": b.shapes(),
           "input_gen_s": t_gen, "workspace_GB": b.workspace.numel() / 1e9}
    b.close()
    return out


def cpu_baseline(corpus, queries, pi, N, k, nq, nq_single=16):
    """The CPU oracle (plain C, OpenMP over rows) on a bounded sample, on all
    the host cores it may use and on one thread."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    used = oracle.set_threads(threads)
    t = time.perf_counter()
    S = oracle.sketch_sets(corpus.indptr, corpus.indices, corpus.d, pi, N)
    oracle.pack(S, N)
    t_sk = time.perf_counter() - t
    SQ = oracle.sketch_sets(queries.indptr, queries.indices, queries.d, pi, N)
    sub = oracle.Sets(SQ.vals, SQ.start[:nq], SQ.length[:nq])
    t = time.perf_counter()
    oracle.topk(sub, S, N, oracle.JS, k)
    t_tk = time.perf_counter() - t
    pairs = nq * corpus.n
    # one thread, on fewer queries
    oracle.set_threads(1)
    sub1 = oracle.Sets(SQ.vals, SQ.start[:nq_single], SQ.length[:nq_single])
    t = time.perf_counter()
    oracle.topk(sub1, S, N, oracle.JS, k)
    t_1 = time.perf_counter() - t
    t = time.perf_counter()
    S1 = oracle.sketch_sets(corpus.indptr, corpus.indices, corpus.d, pi, N)
    oracle.pack(S1, N)
    t_sk1 = time.perf_counter() - t
    oracle.set_threads(threads)
    return {"value": pairs / t_tk, "unit": "pair estimates/s", "cores": used, "kind": "oracle",
            "sample": "oracle top-%d Jaccard of %d queries x %d corpus rows at N=%d (%.1f s); "
                      "oracle sketch of all %d corpus rows (%.2f s)" % (
                          k, nq, corpus.n, N, t_tk, corpus.n, t_sk),
            "sketch_vectors_per_s": corpus.n / t_sk,
            "single_thread": {"value": nq_single * corpus.n / t_1, "unit": "pair estimates/s", "cores": 1,
                              "sample": "oracle top-%d Jaccard of %d queries x %d corpus rows at N=%d (%.1f s); "
                                        "oracle sketch of all %d corpus rows (%.2f s)" % (
                                            k, nq_single, corpus.n, N, t_1, corpus.n, t_sk1),
                              "sketch_vectors_per_s": corpus.n / t_sk1}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--other-widths", default="256,4096", help="extra widths reported (empty: none)")
    ap.add_argument("--cpu-queries", type=int, default=256, help="queries in the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mse", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-estimator evaluation")
    ap.add_argument("--no-ranking", action="store_true", help="skip the threshold-retrieval evaluation")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems run")
    ap.add_argument("--no-dense", action="store_true", help="skip the small-corpus all-pairs estimate run")
    ap.add_argument("--graph", action="store_true", help="time replays of the step recorded into a HIP graph")
    ap.add_argument("--no-vector-scan", action="store_true",
                    help="skip the extra run of the step with the pair counts on the vector ALU")
    ap.add_argument("--vector-scan", action="store_true",
                    help="count pairs on the vector ALU at every width (profiling the VALU scan; the default puts "
                         "widths that are multiples of 256 on the matrix cores)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--ingest-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_BYTES"),
                    help="write profiles/traffic.json from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of "
                         "`bench.py --other-widths ''` (each directory also holding the copy calibration)")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters, N=args.N)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build runs the hot path on a single MI355X "
              "(requested --gpus %d, WORLD_SIZE %d)." % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_bytes:
        x = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device=dev).fill_(1)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("copied %d bytes" % args.copy_bytes)
        return
    others = [int(x) for x in args.other_widths.split(",") if x.strip()]
    widths = [args.N] + [n for n in others if n != args.N]
    corpus, queries, pis, dev_in = make_inputs(widths, dev)
    nC, nQ, k = corpus.n, queries.n, args.k
    if args.vector_scan:
        from paper_1910_04658_amd import binding as bs
        bs.debug_set_topk_mma(False)

    results = {}
    for i, N in enumerate(widths):
        step = Step(dev_in, N, k, nC, nQ, dev)
        steps = args.steps if i == 0 else max(10, args.steps // 4)
        ms, kt = timed(step, steps, args.warmup, graph=args.graph)
        results[N] = (step, ms, kt, steps)
        log("N=%d: %.4f ms/step; kernels %s" % (N, ms, {n: round(v["avg_ms"], 4) for n, v in kt.items()}))

    step, ms, kt, steps = results[args.N]
    pairs = nQ * nC
    value = pairs / (ms / 1e3)

    def scan_roofline(N, kt):
        from paper_1910_04658_amd import binding as bs
        S = bs.topk_sample_size(nC)  # rows scored by the sample pass, not the scan
        if "topk_scan" not in kt:
            return None
        t = kt["topk_scan"]["avg_ms"] / 1e3
        if N % 256 == 0 and not args.vector_scan:
            # matrix-core scan: x_ab of every scanned pair is an N-term 0/1
            # product, 2 N flops on FP4 operands
            fl = 2 * nQ * (nC - S) * N
            ach = fl / t / 1e12
            return {"bound": "mfma", "achieved": ach, "peak": PEAK_FP4_TFLOPS, "unit": "TFLOP/s",
                    "frac": ach / PEAK_FP4_TFLOPS, "traffic": traffic_for("topk_scan", "N%d" % N),
                    "kernel": "topk_scan", "flops_per_launch": fl, "avg_launch_ms": kt["topk_scan"]["avg_ms"]}
        ops = nQ * (nC - S) * (N // 16)  # one AND and one popcount per 32-bit word pair
        ach = ops / t / 1e12
        return {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                "frac": ach / PEAK_VALU_TOPS, "traffic": traffic_for("topk_scan", "N%d" % N),
                "kernel": "topk_scan", "ops_per_launch": ops, "avg_launch_ms": kt["topk_scan"]["avg_ms"]}

    def sketch_rate(kt):
        # corpus and query rows per second of sketch-kernel time
        t = sum(kt[n]["avg_ms"] * kt[n]["per_step"] for n in ("sketch_pack", "sketch_csr") if n in kt) / 1e3
        return (nC + nQ) / t if t > 0 else None

    def sketch_roofline(N, kt):
        if "sketch_csr" not in kt:
            return None
        # corpus and queries (one launch per step; the time per step in general)
        rows = nC + nQ
        nnz = corpus.nnz + queries.nnz
        by = (rows + 2) * 4 + nnz * 4 + rows * (N // 8) + rows * 4 + corpus.d * 4
        t = kt["sketch_csr"]["avg_ms"] * kt["sketch_csr"]["per_step"] / 1e3
        ach = by / t / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                "traffic": traffic_for("sketch_csr", "N%d" % N), "kernel": "sketch_csr",
                "bytes_per_step": by, "avg_launch_ms": kt["sketch_csr"]["avg_ms"]}

    out = {
        "metric": "sketched vectors/s + pair estimates/s at N=1024; Jaccard MSE vs exact",
        "value": value,
        "unit": "pair estimates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # scores are FP32; the pair counts behind them are exact integers (0/1
        # FP4 matrix-core operands with FP32 accumulators, or VALU popcounts)
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "BinSketch sketch + top-100 Jaccard query-vs-corpus", "N": args.N,
                   "n_corpus": nC, "n_queries": nQ, "d": corpus.d, "k": k,
                   "row_length": "round(lognormal), mean 230, sd 150",
                   "feature_popularity": "Zipf(1.1)", "score_dtype": "f32",
                   "pair_counts": ("exact integers: VALU AND + popcount at every width (--vector-scan)"
                                   if args.vector_scan else
                                   "exact integers: 0/1 FP4 matrix-core operands with FP32 accumulators "
                                   "(N a multiple of 256), else VALU AND + popcount"), "parallelism": "single GPU"},
        "sketched_vectors_per_s": sketch_rate(kt),
        "pair_estimates_per_s": value,
        "kernels_ms": {n: v["avg_ms"] for n, v in kt.items()},
        "roofline": scan_roofline(args.N, kt),
        "roofline_sketch": sketch_roofline(args.N, kt),
    }
    out["widths"] = {}
    for N in widths:
        if N == args.N:
            continue
        st, msN, ktN, stepsN = results[N]
        out["widths"][str(N)] = {"ms_per_step": msN, "pair_estimates_per_s": pairs / (msN / 1e3),
                                 "sketched_vectors_per_s": sketch_rate(ktN),
                                 "kernels_ms": {n: v["avg_ms"] for n, v in ktN.items()},
                                 "roofline": scan_roofline(N, ktN), "roofline_sketch": sketch_roofline(N, ktN)}
    if not args.no_mse:
        out["jaccard_mse"] = {str(N): jaccard_mse(results[N][0], corpus, queries) for N in widths}
    if not args.vector_scan and not args.no_vector_scan and args.N % 256 == 0:
        # the same step with the pair counts on the vector ALU (AND + popcount),
        # for the int32 VALU roofline of the popcount path at the metric's width
        from paper_1910_04658_amd import binding as bs
        bs.debug_set_topk_mma(False)
        try:
            vstep = Step(dev_in, args.N, k, nC, nQ, dev)
            vms, vkt = timed(vstep, 20, 3)
        finally:
            bs.debug_set_topk_mma(True)
        S = bs.topk_sample_size(nC)
        ops = nQ * (nC - S) * (args.N // 16)
        t = vkt["topk_scan"]["avg_ms"] / 1e3
        out["vector_scan"] = {
            "N": args.N, "ms_per_step": vms, "pair_estimates_per_s": nQ * nC / (vms / 1e3),
            "kernels_ms": {n: v["avg_ms"] for n, v in vkt.items()},
            "roofline": {"bound": "alu", "achieved": ops / t / 1e12, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                         "frac": ops / t / 1e12 / PEAK_VALU_TOPS, "kernel": "topk_scan", "ops_per_launch": ops,
                         "avg_launch_ms": vkt["topk_scan"]["avg_ms"]}}
        log("vector scan: %s" % out["vector_scan"])
    if not args.no_dense:
        log("all-pairs estimates of the small corpus ...")
        out["dense_small_corpus"] = dense_eval(dev)
        log("dense: %s" % out["dense_small_corpus"])
    if not args.no_batch:
        log("batched problems ...")
        out["batching"] = batch_eval(dev)
        log("batching: %s" % out["batching"])
    if not args.no_serving:
        log("serving run ...")
        out["serving"] = serving_eval(dev)
        log("serving: %s" % out["serving"])
    if not args.no_learned:
        log("training the learned estimator ...")
        out["learned_estimator"] = learned_eval(dev)
        log("learned estimator: %s" % out["learned_estimator"])
    if not args.no_ranking:
        log("threshold retrieval (ranking experiment) ...")
        out["ranking"] = ranking_eval(dev)
        log("ranking: %s" % json.dumps(out["ranking"]["widths"].get(str(args.N))))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(corpus, queries, pis[args.N], args.N, k, args.cpu_queries)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
