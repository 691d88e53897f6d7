"""Seeded synthetic inputs for BinSketch: sparse binary corpora in CSR form and
random maps pi:[d] -> [N].

This module holds none of the sketching or estimation arithmetic. It only draws
inputs, and it is the one module that both the CPU oracle's tests and the GPU
path's tests and benchmark use. The random map of the BinSketch definition
(Section 3, Definition "BinSketch": pi is one of the N^d functions from
{1..d} to {1..N}, so every coordinate is mapped independently and uniformly)
is drawn here and handed to both sides as an input table.

Conventions (0-based, where the paper counts from 1):
  * a binary vector a in {0,1}^d is a sorted list of its set indices (the
    sparse representation of Section 1.1), stored row after row in CSR form:
    ``indptr`` int32[n+1], ``indices`` int32[nnz];
  * ``pi`` is int32[d] with values in [0, N).

Generators:
  * ``splitmix64``: Steele, Lea and Flood, "Fast splittable pseudorandom number
    generators" (OOPSLA 2014); the table entry for coordinate i is the i-th
    output of the stream started at ``seed``, reduced to [0, N) by the
    multiply-high map (x >> 32) * N >> 32, which is exactly uniform when N is a
    power of two.
  * row lengths: Zipf(s) truncated to [lo, hi], or a rounded log-normal;
  * feature ids: popularity proportional to rank^-s (Zipf), drawn without
    replacement within a row by successive sampling (draw with replacement,
    keep first occurrences), ranks mapped to ids through a seeded permutation.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream for ``seed``."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def random_map(d: int, N: int, seed: int) -> np.ndarray:
    """pi:[d] -> [N], i.i.d. uniform per coordinate, as int32[d]."""
    if d < 0 or N <= 0:
        raise ValueError("need d >= 0 and N > 0")
    z = splitmix64(seed, d)
    with np.errstate(over="ignore"):
        v = ((z >> np.uint64(32)) * np.uint64(N)) >> np.uint64(32)
    return v.astype(np.int32)


@dataclasses.dataclass
class CSR:
    """A batch of binary vectors: row r has set indices indices[indptr[r]:indptr[r+1]]."""

    indptr: np.ndarray  # int32[n+1]
    indices: np.ndarray  # int32[nnz]
    d: int

    @property
    def n(self) -> int:
        return len(self.indptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, r: int) -> np.ndarray:
        return self.indices[self.indptr[r]:self.indptr[r + 1]]

    def lengths(self) -> np.ndarray:
        return np.diff(self.indptr.astype(np.int64))

    def take(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.lengths()[rows]
        indptr = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        parts = [self.row(int(r)) for r in rows]
        indices = np.concatenate(parts) if parts else np.zeros(0, np.int32)
        return CSR(indptr.astype(np.int32), indices.astype(np.int32), self.d)


def from_rows(rows, d: int) -> CSR:
    """CSR from a list of index sequences (kept as given: order, duplicates)."""
    lens = [len(r) for r in rows]
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    if indptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indptr; split the batch")
    indices = (np.concatenate([np.asarray(r, dtype=np.int64) for r in rows])
               if rows and indptr[-1] > 0 else np.zeros(0, np.int64))
    return CSR(indptr.astype(np.int32), indices.astype(np.int32), d)


def zipf_truncated_lengths(rng: np.random.Generator, n: int, s: float, lo: int, hi: int) -> np.ndarray:
    """n draws of P(m) proportional to m^-s on the integers lo..hi."""
    m = np.arange(lo, hi + 1, dtype=np.float64)
    cdf = np.cumsum(m ** -s)
    cdf /= cdf[-1]
    return (lo + np.searchsorted(cdf, rng.random(n), side="right")).astype(np.int64).clip(lo, hi)


def lognormal_lengths(rng: np.random.Generator, n: int, mean: float, sd: float,
                      lo: int = 1, hi: int | None = None) -> np.ndarray:
    """Rounded log-normal lengths with the given mean and standard deviation."""
    sigma2 = math.log1p((sd / mean) ** 2)
    mu = math.log(mean) - sigma2 / 2
    x = np.rint(rng.lognormal(mu, math.sqrt(sigma2), n)).astype(np.int64)
    return x.clip(lo, hi if hi is not None else np.iinfo(np.int64).max)


def zipf_rows(rng: np.random.Generator, lengths: np.ndarray, d: int, s: float) -> CSR:
    """Rows of the given lengths; ids drawn by Zipf(s) popularity without replacement.

    Popularity of rank r (0-based) is proportional to (r+1)^-s; rank r names the
    id perm[r] for a seeded permutation perm of [0, d). Within a row, draws are
    taken with replacement and only first occurrences are kept, which is exactly
    sampling without replacement proportionally to the remaining weights. Each
    row is returned sorted by id.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    if (lengths > d).any():
        raise ValueError("a row cannot hold more than d distinct ids")
    n = len(lengths)
    perm = rng.permutation(d).astype(np.int64)
    cdf = np.cumsum(np.arange(1, d + 1, dtype=np.float64) ** -s)
    cdf /= cdf[-1]

    chosen = [None] * n
    draws = [np.zeros(0, np.int64) for _ in range(n)]
    pending = np.nonzero(lengths > 0)[0]
    for r in np.nonzero(lengths == 0)[0]:
        chosen[r] = np.zeros(0, np.int64)
    factor = 3.0
    while len(pending):
        want = np.ceil(lengths[pending] * factor).astype(np.int64) + 16
        total = int(want.sum())
        ranks = np.searchsorted(cdf, rng.random(total), side="right").clip(0, d - 1)
        offs = np.zeros(len(pending) + 1, np.int64)
        np.cumsum(want, out=offs[1:])
        still = []
        for j, r in enumerate(pending):
            seq = np.concatenate([draws[r], ranks[offs[j]:offs[j + 1]]])
            _, first = np.unique(seq, return_index=True)
            if len(first) >= lengths[r]:
                keep = np.sort(first)[:lengths[r]]
                chosen[r] = seq[keep]
                draws[r] = None
            else:
                draws[r] = seq
                still.append(r)
        pending = np.asarray(still, dtype=np.int64)
        factor *= 2.0
    rows = [np.sort(perm[c]) for c in chosen]
    return from_rows(rows, d)


def zipf_rows_fast(rng: np.random.Generator, lengths: np.ndarray, d: int, s: float) -> CSR:
    """Vectorised form of :func:`zipf_rows` for large corpora (same distribution).

    All rows draw an oversized batch at once; first occurrences are found with
    one global sort; the few rows left short fall back to :func:`zipf_rows`'s
    per-row loop, continuing their own draw sequence.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    if (lengths > d).any():
        raise ValueError("a row cannot hold more than d distinct ids")
    n = len(lengths)
    perm = rng.permutation(d).astype(np.int64)
    cdf = np.cumsum(np.arange(1, d + 1, dtype=np.float64) ** -s)
    cdf /= cdf[-1]
    want = np.ceil(lengths * 3.0).astype(np.int64) + 16
    want[lengths == 0] = 0
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(want, out=offs[1:])
    total = int(offs[-1])
    ranks = np.searchsorted(cdf, rng.random(total), side="right").clip(0, d - 1).astype(np.int64)
    row_of = np.repeat(np.arange(n, dtype=np.int64), want)
    pos = np.arange(total, dtype=np.int64)
    key = row_of * d + ranks
    order = np.lexsort((pos, key))  # by key, then by draw position
    ks = key[order]
    is_first = np.ones(total, bool)
    is_first[1:] = ks[1:] != ks[:-1]
    fpos = pos[order][is_first]  # draw positions of first occurrences
    fpos.sort()  # grouped by row (positions are row-contiguous), in draw order
    frow = row_of[fpos]
    counts = np.bincount(frow, minlength=n)
    start = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=start[1:])
    rank_in_row = np.arange(len(fpos), dtype=np.int64) - start[frow]
    keep = rank_in_row < lengths[frow]
    kpos = fpos[keep]
    krow = row_of[kpos]
    ids = perm[ranks[kpos]]
    short = np.nonzero(counts < lengths)[0]
    # sort ids within rows
    o = np.lexsort((ids, krow))
    ids, krow = ids[o], krow[o]
    got = np.bincount(krow, minlength=n)
    if len(short):
        # Continue each short row's own draw sequence until it has enough ids.
        extra_rng = rng
        rows_fix = {}
        for r in short:
            seq = ranks[offs[r]:offs[r + 1]]
            while True:
                _, first = np.unique(seq, return_index=True)
                if len(first) >= lengths[r]:
                    break
                seq = np.concatenate([seq, np.searchsorted(
                    cdf, extra_rng.random(int(lengths[r]) * 4 + 16), side="right").clip(0, d - 1)])
            keepi = np.sort(first)[:lengths[r]]
            rows_fix[int(r)] = np.sort(perm[seq[keepi]])
        indptr = np.zeros(n + 1, np.int64)
        np.cumsum(lengths, out=indptr[1:])
        out = np.empty(int(indptr[-1]), np.int64)
        gstart = np.zeros(n + 1, np.int64)
        np.cumsum(got, out=gstart[1:])
        mask_ok = np.ones(n, bool)
        mask_ok[short] = False
        # rows that were complete: copy blocks
        okrows = np.nonzero(mask_ok & (lengths > 0))[0]
        src = np.concatenate([np.arange(gstart[r], gstart[r + 1]) for r in okrows]) if len(okrows) else np.zeros(0, np.int64)
        dst = np.concatenate([np.arange(indptr[r], indptr[r + 1]) for r in okrows]) if len(okrows) else np.zeros(0, np.int64)
        out[dst] = ids[src]
        for r, v in rows_fix.items():
            out[indptr[r]:indptr[r + 1]] = v
        if indptr[-1] >= 2 ** 31:
            raise ValueError("nnz does not fit int32 indptr; split the batch")
        return CSR(indptr.astype(np.int32), out.astype(np.int32), d)
    indptr = np.zeros(n + 1, np.int64)
    np.cumsum(got, out=indptr[1:])
    if indptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indptr; split the batch")
    return CSR(indptr.astype(np.int32), ids.astype(np.int32), d)


# ---------------------------------------------------------------------------
# Workload recipes (sizes and distributions of the benchmark workloads)
# ---------------------------------------------------------------------------

SEED_PI = 0x5EED_B1A5
SEED_SMALL = 1001
SEED_CORPUS = 2002
SEED_QUERIES = 3003


def small_corpus(n: int = 1000, d: int = 10_000, seed: int = SEED_SMALL) -> CSR:
    """n vectors, d dims, lengths Zipf(1.1) truncated to [5, 500], Zipf(1.1) ids."""
    rng = np.random.default_rng(seed)
    lengths = zipf_truncated_lengths(rng, n, 1.1, 5, 500)
    return zipf_rows(rng, lengths, d, 1.1)


def lognormal_corpus(n: int, d: int = 100_000, mean: float = 230.0, sd: float = 150.0,
                     seed: int = SEED_CORPUS, fast: bool = True) -> CSR:
    """n vectors, d dims, lengths round(lognormal) with the given mean/sd (>= 1)."""
    rng = np.random.default_rng(seed)
    lengths = lognormal_lengths(rng, n, mean, sd, lo=1, hi=d)
    gen = zipf_rows_fast if fast else zipf_rows
    return gen(rng, lengths, d, 1.1)


def identity_map(N: int) -> np.ndarray:
    """pi(i) = i on [N]: with d = N every row is its own sketch."""
    return np.arange(N, dtype=np.int32)


def saturation_rows(n: int, N: int, seed: int, p_empty: float = 0.03, p_full: float = 0.03,
                    p_near: float = 0.06, len_hi: int = 4096, last_full: bool = False) -> CSR:
    """n rows over [0, N), meant for the identity map (d = N), so that their
    sketches are chosen directly: a mix of empty rows, full rows (all N
    coordinates), rows missing 1-8 coordinates, and rows whose length is
    log-uniform on [1, min(len_hi, N)] with uniform distinct coordinates.
    The empty and full rows drive the 0/0 and x = N (saturation) cases of the
    estimators; ``last_full`` makes the last row full."""
    rng = np.random.default_rng(seed)
    kind = rng.choice(4, size=n, p=[p_empty, p_full, p_near, 1.0 - p_empty - p_full - p_near])
    if last_full and n > 0:
        kind[-1] = 1
    hi = min(len_hi, N)
    rows = []
    for r in range(n):
        if kind[r] == 0:
            rows.append(np.zeros(0, np.int64))
        elif kind[r] == 1:
            rows.append(np.arange(N, dtype=np.int64))
        elif kind[r] == 2:
            holes = rng.choice(N, size=int(rng.integers(1, 9)), replace=False)
            keep = np.ones(N, bool)
            keep[holes] = False
            rows.append(np.nonzero(keep)[0])
        else:
            m = int(np.exp(rng.uniform(0.0, np.log(hi))))
            rows.append(np.sort(rng.choice(N, size=max(m, 1), replace=False)))
    return from_rows(rows, N)


def planted_pairs(rng: np.random.Generator, base: CSR, frac: np.ndarray, s: float = 1.1) -> CSR:
    """For each row a of ``base``, a partner b = a with a fraction frac[r] of its ids
    replaced by fresh Zipf(s)-popular ids not already in a (near-duplicate pairs)."""
    d = base.d
    cdf = np.cumsum(np.arange(1, d + 1, dtype=np.float64) ** -s)
    cdf /= cdf[-1]
    perm = rng.permutation(d).astype(np.int64)
    rows = []
    for r in range(base.n):
        a = base.row(r).astype(np.int64)
        m = len(a)
        nrep = int(round(frac[r] * m))
        keep = rng.permutation(m)[: m - nrep]
        cur = set(int(x) for x in a)
        kept = [int(a[i]) for i in keep]
        new = []
        while len(new) < nrep and len(cur) < d:
            cand = perm[np.searchsorted(cdf, rng.random(2 * nrep + 8), side="right").clip(0, d - 1)]
            for c in cand:
                c = int(c)
                if c not in cur:
                    cur.add(c)
                    new.append(c)
                    if len(new) == nrep:
                        break
        rows.append(np.sort(np.asarray(kept + new, dtype=np.int64)))
    return from_rows(rows, d)


# ---------------------------------------------------------------------------
# Pairs with known Jaccard similarity (training data for a learned estimator)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PairSet:
    """Vectors (CSR) and index pairs into them with their exact Jaccard similarity."""

    csr: CSR
    ia: np.ndarray      # int32[n_pairs]
    ib: np.ndarray      # int32[n_pairs]
    inter: np.ndarray   # int32[n_pairs] |a n b|
    jaccard: np.ndarray  # float64[n_pairs] |a n b| / |a u b| (0 for two empty sets)


def variant_groups(n_groups: int, group_size: int, d: int = 100_000, mean: float = 230.0, sd: float = 150.0,
                   s: float = 1.1, seed: int = 4004) -> PairSet:
    """Groups of near-duplicate vectors and all pairs inside each group.

    Each group starts from a base vector (row lengths round(lognormal(mean, sd)),
    Zipf(s) ids, as `lognormal_corpus`). Each of its `group_size` members keeps
    every base id with probability 1 - f and adds round(f * |base|) fresh
    Zipf(s) ids, f ~ U(0, 1) drawn per member, so pair similarities cover [0, 1].
    Every unordered pair of members of a group is listed, with its exact
    intersection size and Jaccard similarity (set arithmetic on the ids).
    """
    rng = np.random.default_rng(seed)
    base = lognormal_corpus(n_groups, d=d, mean=mean, sd=sd, seed=int(rng.integers(1 << 62)))
    G = group_size
    blen = base.lengths()
    cdf = np.cumsum(np.arange(1, d + 1, dtype=np.float64) ** -s)
    cdf /= cdf[-1]
    perm = rng.permutation(d).astype(np.int64)
    n_mem = n_groups * G
    f = rng.random(n_mem)
    mem_group = np.repeat(np.arange(n_groups), G)
    # kept base ids
    reps = blen[mem_group]
    starts = base.indptr[:-1].astype(np.int64)[mem_group]
    off = np.arange(int(reps.sum()), dtype=np.int64) - np.repeat(np.cumsum(reps) - reps, reps)
    kept_ids = base.indices.astype(np.int64)[np.repeat(starts, reps) + off]
    kept_mem = np.repeat(np.arange(n_mem), reps)
    keep = rng.random(len(kept_ids)) >= np.repeat(f, reps)
    # fresh ids
    n_new = np.rint(f * blen[mem_group]).astype(np.int64)
    new_ids = perm[np.searchsorted(cdf, rng.random(int(n_new.sum())), side="right").clip(0, d - 1)]
    new_mem = np.repeat(np.arange(n_mem), n_new)
    mem = np.concatenate([kept_mem[keep], new_mem])
    ids = np.concatenate([kept_ids[keep], new_ids])
    key = np.unique(mem * d + ids)
    mem_u = key // d
    ids_u = (key % d).astype(np.int32)
    counts = np.bincount(mem_u, minlength=n_mem)
    indptr = np.zeros(n_mem + 1, np.int64)
    np.cumsum(counts, out=indptr[1:])
    if indptr[-1] >= 2 ** 31:
        raise ValueError("too many set bits for one int32 CSR batch")
    csr = CSR(indptr.astype(np.int32), ids_u, d)
    # exact intersections inside each group: dense 0/1 matrix over the group's ids
    iu, ju = np.triu_indices(G, 1)
    ia = np.empty(n_groups * len(iu), np.int32)
    ib = np.empty_like(ia)
    inter = np.empty_like(ia)
    for g in range(n_groups):
        lo, hi = indptr[g * G], indptr[(g + 1) * G]
        local, inv = np.unique(ids_u[lo:hi], return_inverse=True)
        M = np.zeros((G, len(local)), np.float32)
        M[np.repeat(np.arange(G), counts[g * G:(g + 1) * G]), inv] = 1.0
        I = M @ M.T
        sl = slice(g * len(iu), (g + 1) * len(iu))
        ia[sl] = g * G + iu
        ib[sl] = g * G + ju
        inter[sl] = I[iu, ju].astype(np.int32)
    la = counts[ia].astype(np.float64)
    lb = counts[ib].astype(np.float64)
    union = la + lb - inter
    jac = np.where(union > 0, inter / np.maximum(union, 1), 0.0)
    return PairSet(csr, ia, ib, inter, jac)


# ---------------------------------------------------------------------------
# Large corpora generated on the device, chunk by chunk (serving workload)
# ---------------------------------------------------------------------------

def device_corpus_chunks(n: int, d: int, mean: float, sd: float, seed: int, device, chunk_rows: int = 1 << 18,
                         s: float = 1.1, lo: int = 1, hi: int | None = None):
    """Yields (indptr int32[m+1], indices int32[nnz]) device tensors for
    consecutive chunks of an n-row corpus: lengths round(lognormal(mean, sd))
    clipped to [lo, hi], ids drawn by Zipf(s) popularity *with* replacement
    (a row may repeat an id; the binary vector is the set of its ids), ranks
    mapped to ids by a seeded permutation. Uses torch's device generator only
    to draw random numbers; nothing of the method is computed here."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cdf = torch.cumsum(torch.arange(1, d + 1, device=device, dtype=torch.float64) ** -s, 0)
    cdf /= cdf[-1].clone()
    perm = torch.randperm(d, generator=g, device=device)
    sigma2 = math.log1p((sd / mean) ** 2)
    mu = math.log(mean) - sigma2 / 2
    hi = hi if hi is not None else d
    for r0 in range(0, n, chunk_rows):
        m = min(chunk_rows, n - r0)
        z = torch.randn(m, generator=g, device=device, dtype=torch.float64)
        lens = torch.exp(mu + math.sqrt(sigma2) * z).round().clamp(lo, hi).to(torch.int64)
        indptr = torch.zeros(m + 1, dtype=torch.int64, device=device)
        torch.cumsum(lens, 0, out=indptr[1:])
        nnz = int(indptr[-1].item())
        if nnz >= 2 ** 31:
            raise ValueError("chunk too large for an int32 CSR batch; lower chunk_rows")
        u = torch.rand(nnz, generator=g, device=device, dtype=torch.float64)
        ranks = torch.searchsorted(cdf, u).clamp_max(d - 1)
        yield indptr.to(torch.int32), perm[ranks].to(torch.int32)


SEED_RANKING = 5005


def concat_rows(a: CSR, b: CSR) -> CSR:
    """The rows of a, then the rows of b (same dimension)."""
    if a.d != b.d:
        raise ValueError("dimensions differ")
    indptr = np.concatenate([a.indptr[:-1].astype(np.int64), b.indptr.astype(np.int64) + a.nnz])
    if indptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indptr; split the batch")
    return CSR(indptr.astype(np.int32), np.concatenate([a.indices, b.indices]).astype(np.int32), a.d)


def ranking_split(n_background: int = 20_000, n_groups: int = 1000, group_size: int = 10, d: int = 100_000,
                  seed: int = SEED_RANKING, query_frac: float = 0.1):
    """Data of the ranking experiment (Section 4.2, Experiment 2) on synthetic
    rows: `n_background` rows of the benchmark distribution plus `n_groups`
    groups of `group_size` near-duplicates (variant_groups), so that exact
    similarities reach the high thresholds, shuffled and split into a
    corpus (1 - query_frac of the rows) and queries, the queries in random
    order (so any prefix is a random sample). Returns (corpus, queries)."""
    rng = np.random.default_rng(seed)
    bg = lognormal_corpus(n_background, d=d, seed=int(rng.integers(1 << 62)))
    gr = variant_groups(n_groups, group_size, d=d, seed=int(rng.integers(1 << 62))).csr
    rows = concat_rows(bg, gr)
    perm = rng.permutation(rows.n)
    nq = int(round(query_frac * rows.n))
    return rows.take(np.sort(perm[nq:])), rows.take(perm[:nq])


def loguniform_lengths(rng: np.random.Generator, n: int, lo: int, hi: int) -> np.ndarray:
    """Integer lengths with log-uniform distribution on [lo, hi]."""
    return np.exp(rng.uniform(math.log(lo), math.log(hi + 1), n)).astype(np.int64).clip(lo, hi)


def serving_queries(n: int, d: int, seed: int, lo: int = 10, hi: int = 5000, rate: float = 2000.0):
    """n query vectors (log-uniform lengths in [lo, hi], Zipf(1.1) ids without
    replacement) and Poisson arrival times (seconds) at `rate` queries/s."""
    rng = np.random.default_rng(seed)
    lens = loguniform_lengths(rng, n, lo, hi)
    q = zipf_rows_fast(rng, lens, d, 1.1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n)) if rate > 0 else np.zeros(n)
    return q, arrivals


# ---- batches of uneven problems -------------------------------------------------
SEED_BATCH = 4004
BATCH_WIDTHS = (128, 512, 2048, 8192)


@dataclasses.dataclass
class BatchSpec:
    n: int        # corpus rows
    d: int        # dimension
    mean: float   # mean set bits per row
    N: int        # sketch width
    nq: int       # query rows
    seed: int


def batch_specs(n_problems: int = 64, seed: int = SEED_BATCH, n_lo: int = 1000, n_hi: int = 200_000,
                d_lo: int = 10_000, d_hi: int = 1_000_000, m_lo: float = 20.0, m_hi: float = 2000.0,
                widths=BATCH_WIDTHS, q_frac: float = 0.01, q_min: int = 100) -> list:
    """Shapes of a batch of independent problems: corpus size, dimension and
    mean row weight each log-uniform (a power law with exponent -1) on their
    ranges, the width uniform over `widths`, queries q_frac of the rows (at
    least q_min)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_problems):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(round(math.exp(rng.uniform(math.log(d_lo), math.log(d_hi)))))
        mean = float(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi))))
        N = int(widths[int(rng.integers(len(widths)))])
        nq = max(q_min, int(round(q_frac * n)))
        out.append(BatchSpec(n, d, mean, N, nq, seed * 1000 + i))
    return out


def device_batch(specs: list, device, k: int = 100, cv: float = 0.65) -> list:
    """Device tensors of every problem of a batch: corpus and query CSR (row
    lengths lognormal with the spec's mean and sd = cv * mean, clipped to
    [1, min(d, 10 * mean)]; ids by Zipf(1.1) popularity with replacement), the
    map pi and the problem's N, d and k (k capped at the corpus size)."""
    import torch
    probs = []
    for sp in specs:
        hi = int(min(sp.d, max(2, 10 * sp.mean)))
        parts = []
        for rows, sd_seed in ((sp.n, sp.seed), (sp.nq, sp.seed + 7919)):
            if rows == 0:
                parts.append((torch.zeros(1, dtype=torch.int32, device=device),
                              torch.zeros(0, dtype=torch.int32, device=device)))
                continue
            (ip, ix), = list(device_corpus_chunks(rows, sp.d, sp.mean, cv * sp.mean, sd_seed, device,
                                                  chunk_rows=rows, hi=hi))
            parts.append((ip, ix))
        pi = torch.from_numpy(random_map(sp.d, sp.N, SEED_PI + sp.seed)).to(device)
        probs.append({"indptr": parts[0][0], "indices": parts[0][1], "q_indptr": parts[1][0],
                      "q_indices": parts[1][1], "pi": pi, "d": sp.d, "N": sp.N, "k": min(k, sp.n)})
    return probs
