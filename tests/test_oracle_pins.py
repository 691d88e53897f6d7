"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: a
definition evaluated coordinate by coordinate, exhaustive enumeration of every
random map, Monte-Carlo against Lemma 1's closed forms, inversion of Lemma 1 by
Algorithm 1, dense linear algebra, brute-force sorting, and special cases.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows_csr(rows, d):
    c = datagen.from_rows(rows, d)
    return c.indptr, c.indices


def _bits_from_words(words, N):
    w = np.asarray(words, dtype=np.uint64)
    return [int((int(w[j // 64]) >> (j % 64)) & 1) for j in range(N)]


# --- the sketch: Section 3, Definition "BinSketch" --------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_sketch_equals_definition_coordinatewise(seed):
    """Packed oracle sketch == OR over each preimage pi^-1(j), evaluated for every j."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 60))
    N = int(rng.choice([64, 128, 192]))
    pi = rng.integers(0, N, d).astype(np.int32)
    rows = [rng.choice(d, int(rng.integers(0, d + 1)), replace=False) for _ in range(5)]
    ip, ix = _rows_csr(rows, d)
    words, pop = oracle.sketch(ip, ix, d, pi, N)
    for r, row in enumerate(rows):
        a_bits = [0] * d
        for i in row:
            a_bits[int(i)] = 1
        ref = oracle.sketch_by_definition(a_bits, pi, N)
        assert _bits_from_words(words[r], N) == ref
        assert pop[r] == sum(ref)


def test_sketch_invariants():
    rng = np.random.default_rng(11)
    d, N = 500, 128
    pi = rng.integers(0, N, d).astype(np.int32)
    for _ in range(50):
        a = rng.choice(d, int(rng.integers(0, 200)), replace=False)
        b = rng.choice(d, int(rng.integers(0, 200)), replace=False)
        u = np.union1d(a, b)
        sub = a[: len(a) // 2]
        ip, ix = _rows_csr([a, b, u, sub], d)
        w, pop = oracle.sketch(ip, ix, d, pi, N)
        # popcount(a_s) <= min(N, |a|)
        assert pop[0] <= min(N, len(a)) and pop[1] <= min(N, len(b))
        # the sketch of a union is the OR of the sketches
        assert np.array_equal(w[2], w[0] | w[1])
        # a subset's sketch is a subset of the sketch
        assert np.array_equal(w[3] & w[0], w[3])


def test_identity_map_reproduces_vector():
    d = N = 128
    pi = np.arange(d, dtype=np.int32)
    rng = np.random.default_rng(3)
    a = np.sort(rng.choice(d, 40, replace=False))
    ip, ix = _rows_csr([a], d)
    w, pop = oracle.sketch(ip, ix, d, pi, N)
    assert _bits_from_words(w[0], N) == [1 if j in set(a.tolist()) else 0 for j in range(N)]
    assert pop[0] == 40


def test_duplicates_and_order_do_not_change_sketch():
    rng = np.random.default_rng(5)
    d, N = 300, 256
    pi = rng.integers(0, N, d).astype(np.int32)
    a = rng.choice(d, 80, replace=False)
    messy = np.concatenate([a[::-1], a[:20], a[5:9]])
    ip, ix = _rows_csr([np.sort(a), messy], d)
    w, pop = oracle.sketch(ip, ix, d, pi, N)
    assert np.array_equal(w[0], w[1]) and pop[0] == pop[1]


def test_malformed_inputs_raise():
    pi = np.zeros(10, np.int32)
    ip, ix = _rows_csr([[1, 2, 10]], 10)
    with pytest.raises(ValueError):
        oracle.sketch(ip, ix, 10, pi, 64)
    ip, ix = _rows_csr([[1, 2]], 10)
    pi_bad = np.full(10, 64, np.int32)
    with pytest.raises(ValueError):
        oracle.sketch(ip, ix, 10, pi_bad, 64)


# --- Lemma 1 by exhaustive enumeration -------------------------------------------

def _lemma1(d, N, a, b):
    n = Fraction(N - 1, N)
    A, B, I = len(a), len(b), len(set(a) & set(b))
    e_a = N * (1 - n ** A)
    e_ab_minus = N * (1 - n ** A - n ** B + n ** (A + B - I))
    e_ab_plus = N * (1 - n ** A - n ** B + n ** (A + B + I))
    # the factored middle form of Lemma 1, part 2
    e_ab_mid = N * ((1 - n ** A) * (1 - n ** B) + n ** (A + B) * ((1 / n) ** I - 1))
    return e_a, e_ab_minus, e_ab_plus, e_ab_mid


def test_lemma1_golden_enumeration():
    """Stored exhaustive averages (tests/golden) equal Lemma 1 with the -IP exponent;
    the +IP exponent printed on the last line of the lemma does not match them."""
    doc = json.load(open(os.path.join(HERE, "golden", "lemma1_enumeration.json")))
    for c in doc["cases"]:
        e_a, e_minus, e_plus, e_mid = _lemma1(c["d"], c["N"], c["a"], c["b"])
        assert Fraction(c["E_pop_a"]) == e_a
        assert Fraction(c["E_and_ab"]) == e_minus == e_mid
        if len(set(c["a"]) & set(c["b"])) > 0:
            assert Fraction(c["E_and_ab"]) != e_plus


def test_lemma1_fresh_enumeration():
    """The oracle, enumerated afresh, reproduces the closed forms."""
    for d, N, a, b in [(5, 3, [0, 1, 2], [1, 2, 3, 4]), (4, 3, [0, 1, 2, 3], [0, 1, 2, 3]),
                       (4, 4, [], [0, 1]), (5, 2, [0, 1], [2, 3, 4])]:
        ea, eab = oracle.enumerate_expectations(d, N, a, b)
        e_a, e_minus, _, _ = _lemma1(d, N, a, b)
        assert ea == e_a and eab == e_minus


def test_lemma1_golden_matches_fresh_enumeration():
    doc = json.load(open(os.path.join(HERE, "golden", "lemma1_enumeration.json")))
    c = doc["cases"][0]
    ea, eab = oracle.enumerate_expectations(c["d"], c["N"], c["a"], c["b"])
    assert (ea, eab) == (Fraction(c["E_pop_a"]), Fraction(c["E_and_ab"]))


# --- Lemma 1 by Monte-Carlo over random maps --------------------------------------

def test_lemma1_monte_carlo():
    """Mean |a_s| and <a_s,b_s> over many maps: within 4 standard errors of Lemma 1;
    the sample variance of |a_s| matches the occupancy variance."""
    rng = np.random.default_rng(7)
    d, N = 400, 256
    a = np.arange(0, 150)
    b = np.arange(100, 260)  # |a n b| = 50
    trials = 4000
    pis = rng.integers(0, N, (trials, d)).astype(np.int32)
    xa = np.zeros(trials)
    xab = np.zeros(trials)
    ip, ix = _rows_csr([a, b], d)
    for t in range(trials):
        s = oracle.sketch_sets(ip, ix, d, pis[t], N)
        xa[t] = s.length[0]
        sa = oracle.Sets(s.row(0), [0], [s.length[0]])
        sb = oracle.Sets(s.row(1), [0], [s.length[1]])
        xab[t] = oracle.intersections(sa, sb)[0, 0]
    n = 1 - 1 / N
    m = len(a)
    e_a = N * (1 - n ** m)
    var_a = N * n ** m + N * (N - 1) * (1 - 2 / N) ** m - N * N * n ** (2 * m)
    assert abs(xa.mean() - e_a) < 4 * math.sqrt(var_a / trials)
    assert abs(xa.var(ddof=1) / var_a - 1) < 0.15
    e_ab = N * (1 - n ** 150 - n ** 160 + n ** (150 + 160 - 50))
    assert abs(xab.mean() - e_ab) < 4 * xab.std(ddof=1) / math.sqrt(trials)


def test_lemma2_concentration_failure_rate():
    """Lemma 2: | |a_s| - E|a_s| | < sqrt(psi/2 ln(2/delta)) fails with probability <= delta."""
    rng = np.random.default_rng(9)
    d, N, psi, delta = 300, 512, 100, 0.05
    a = np.arange(psi)
    ip, ix = _rows_csr([a], d)
    bound = math.sqrt(psi / 2 * math.log(2 / delta))
    e_a = N * (1 - (1 - 1 / N) ** psi)
    fails = 0
    trials = 2000
    for _ in range(trials):
        pi = rng.integers(0, N, d).astype(np.int32)
        _, pop = oracle.sketch(ip, ix, d, pi, N)
        fails += abs(pop[0] - e_a) >= bound
    assert fails / trials <= delta


def test_lemma3_concentration_failure_rate():
    """Lemma 3: |<a_s, b_s> - E<a_s, b_s>| < sqrt(psi/2 ln(2/delta)) fails with
    probability at most delta, for |a|, |b| <= psi. The expectation is Lemma 1
    part 2 with the -IP exponent; the +IP exponent printed on its last line
    puts the mean outside the bound in almost every trial."""
    rng = np.random.default_rng(10)
    d, N, psi, delta = 400, 256, 100, 0.05
    a = np.arange(0, 100)
    b = np.arange(60, 160)  # |a n b| = 40
    ip, ix = _rows_csr([a, b], d)
    bound = math.sqrt(psi / 2 * math.log(2 / delta))
    n = 1 - 1 / N
    e_minus = N * (1 - 2 * n ** 100 + n ** (200 - 40))
    e_plus = N * (1 - 2 * n ** 100 + n ** (200 + 40))
    fails = fails_plus = 0
    trials = 2000
    for _ in range(trials):
        pi = rng.integers(0, N, d).astype(np.int32)
        S = oracle.sketch_sets(ip, ix, d, pi, N)
        x = int(oracle.intersections(S, S)[0, 1])
        fails += abs(x - e_minus) >= bound
        fails_plus += abs(x - e_plus) >= bound
    assert fails / trials <= delta
    assert fails_plus / trials > 0.9


# --- the random map: uniform over the N^d functions (Definition BinSketch) ---------

@pytest.mark.parametrize("N,seed", [(64, 1), (1024, 2), (4096, 3)])
def test_random_map_is_uniform(N, seed):
    """Chi-square tests of the map generator: the values of pi are uniform on
    [0, N) and consecutive coordinates are independent (pairs uniform on
    [0, N)^2 for the low 5 bits), as a map drawn uniformly from the N^d
    functions must be."""
    from scipy.stats import chi2
    d = 100 * N
    pi = datagen.random_map(d, N, seed)
    assert pi.dtype == np.int32 and pi.min() >= 0 and pi.max() < N
    cnt = np.bincount(pi, minlength=N)
    e = d / N
    stat = float(((cnt - e) ** 2 / e).sum())
    p = chi2.sf(stat, N - 1)
    assert 1e-4 < p < 1 - 1e-4, (stat, p)
    lo = (pi & 31).astype(np.int64)
    cells = np.bincount(lo[0::2] * 32 + lo[1::2], minlength=1024)
    e2 = (d // 2) / 1024
    stat2 = float(((cells - e2) ** 2 / e2).sum())
    p2 = chi2.sf(stat2, 1023)
    assert 1e-4 < p2 < 1 - 1e-4, (stat2, p2)


# --- Algorithm 1-4: the estimators ------------------------------------------------

def test_algorithm1_inverts_lemma1():
    """Feeding Lemma 1's expectations into Algorithm 1 returns |a|, |b| and IP;
    Algorithms 2-4 then return the exact Ham, JS and Cos."""
    rng = np.random.default_rng(1)
    for _ in range(300):
        N = int(rng.choice([128, 256, 1024, 4096]))
        A = int(rng.integers(1, N // 3))
        B = int(rng.integers(1, N // 3))
        I = int(rng.integers(0, min(A, B) + 1))
        n = 1 - 1 / N
        xa = N * (1 - n ** A)
        xb = N * (1 - n ** B)
        xab = N * (1 - n ** A - n ** B + n ** (A + B - I))
        est = oracle.estimate_literal(xa, xb, xab, N)
        exact = oracle.exact_measures(A, B, I)
        np.testing.assert_allclose(est, exact, rtol=1e-8, atol=1e-7)


def test_canonical_equals_literal_when_unsaturated():
    rng = np.random.default_rng(2)
    for _ in range(2000):
        N = int(rng.choice([64, 256, 1024, 8192]))
        xa = int(rng.integers(0, N))
        xb = int(rng.integers(0, N))
        lo = max(0, xa + xb - (N - 1))
        xab = int(rng.integers(lo, min(xa, xb) + 1))
        if xa == 0 or xb == 0:
            continue
        lit = oracle.estimate_literal(xa, xb, xab, N)
        can = oracle.estimate(xa, xb, xab, N)
        np.testing.assert_allclose(can, lit, rtol=1e-9, atol=1e-9 * max(1.0, abs(lit[0]), abs(lit[1])))


def test_canonical_known_value():
    # N = 1024, (x_a, x_b, x_ab) = (300, 200, 50): computed by hand from the
    # union form with T(x) = ln(1 - x/N) / ln(1 - 1/N).
    N = 1024
    T = lambda x: math.log(1 - x / N) / math.log(1 - 1 / N)  # noqa: E731
    want = T(300) + T(200) - T(450)
    assert abs(want - (-15.2099460950)) < 1e-9
    assert abs(oracle.estimate(300, 200, 50, N)[0] - want) < 1e-9


def test_special_cases():
    N = 1024
    for x in [1, 10, 300, 1000]:
        e = oracle.estimate(x, x, x, N)  # a_s = b_s
        assert abs(e[1]) < 1e-9 and abs(e[2] - 1) < 1e-12 and abs(e[3] - 1) < 1e-12
    T = lambda x: math.log(1 - x / N) / math.log(1 - 1 / N)  # noqa: E731
    e = oracle.estimate(100, 200, 0, N)  # disjoint sketches
    assert e[0] < 0 and abs(e[0] - (T(100) + T(200) - T(300))) < 1e-9
    assert np.all(oracle.estimate(0, 0, 0, N) == 0)
    assert oracle.estimate(0, 50, 0, N)[2] == 0 and oracle.estimate(0, 50, 0, N)[3] == 0


def test_saturation_rule():
    """Counts equal to N are clamped to N-1: outputs stay finite, and a full sketch
    a_s carries only b's size: n_ab = T(x_b)."""
    N = 256
    T = lambda x: math.log(1 - x / N) / math.log(1 - 1 / N)  # noqa: E731
    for xb in [0, 1, 100, 255]:
        e = oracle.estimate(N, xb, xb, N)
        assert np.all(np.isfinite(e))
        assert abs(e[0] - (T(xb) if xb else 0.0)) < 1e-9
    e = oracle.estimate(N, N, N, N)
    assert np.all(np.isfinite(e)) and abs(e[2] - 1) < 1e-12


def test_estimate_pairs_planes_and_strides():
    """The dense FP64 form writes plane m, row p, column q of a [4][nA][nB]
    array with the per-pair canonical estimate of (x_a[p], x_b[q], x_ab[p][q]);
    a non-square shape with counts that differ in every row and column exposes a
    swapped plane, row or stride. Unsaturated pairs also match Algorithm 1 as
    printed (with the Hamming factor 2)."""
    rng = np.random.default_rng(17)
    N, nA, nB = 1024, 37, 53
    xa = rng.integers(0, N + 1, nA).astype(np.int32)
    xb = rng.integers(0, N + 1, nB).astype(np.int32)
    xa[:3] = [0, N, N - 1]
    xb[:3] = [N, 0, 1]
    lo = np.maximum(0, xa[:, None] + xb[None, :] - N)
    hi = np.minimum(xa[:, None], xb[None, :])
    xab = (lo + (rng.random((nA, nB)) * (hi - lo + 1)).astype(np.int64)).astype(np.int32)
    out = oracle.estimate_pairs(xa, xb, xab, N)
    assert out.shape == (4, nA, nB)
    for p in range(nA):
        for q in range(nB):
            ref = oracle.estimate(xa[p], xb[q], xab[p, q], N)
            assert np.array_equal(out[:, p, q], ref), (p, q)
            if 0 < xa[p] < N and 0 < xb[q] < N and xa[p] + xb[q] - xab[p, q] < N:
                lit = oracle.estimate_literal(xa[p], xb[q], xab[p, q], N)
                np.testing.assert_allclose(out[:, p, q], lit, rtol=1e-9,
                                           atol=1e-9 * max(1.0, abs(lit[0]), abs(lit[1])))


def test_score_f32_tracks_fp64():
    rng = np.random.default_rng(4)
    for _ in range(500):
        N = int(rng.choice([256, 1024, 4096]))
        xa, xb = (int(v) for v in rng.integers(1, N, 2))
        xab = int(rng.integers(max(0, xa + xb - N), min(xa, xb) + 1))
        ref = oracle.estimate(xa, xb, xab, N)
        T = lambda x: math.log(1 - min(x, N - 1) / N) / math.log(1 - 1 / N)  # noqa: E731
        Ta, Tb, Tu = T(xa), T(xb), T(xa + xb - xab)
        # FP32 rounding of the three table values and of four operations: a few
        # units of 2^-24 of the magnitudes that cancel in ip = Ta + Tb - Tu
        err_ip = 8 * 2.0 ** -24 * (Ta + Tb + Tu)
        tol = [err_ip, 3 * err_ip, err_ip / (Ta + Tb - ref[0]) + 1e-6,
               err_ip / math.sqrt(Ta * Tb) + 1e-6]
        for m in range(4):
            s = float(oracle.score_f32(xa, xb, xab, N, m))
            assert abs(s - ref[m]) <= tol[m]


# --- exact similarities and ranking ----------------------------------------------

def test_exact_similarities_against_dense_linear_algebra():
    c = datagen.small_corpus(n=200, d=2000, seed=12)
    S = oracle.normalize(c.indptr, c.indices, c.d)
    inter = oracle.intersections(S, S)
    dense = np.zeros((c.n, c.d), np.float64)
    for r in range(c.n):
        dense[r, c.row(r)] = 1
    ip = dense @ dense.T
    assert np.array_equal(inter, ip.astype(np.int32))
    sizes = dense.sum(1)
    for p, q in [(0, 1), (3, 3), (10, 50), (199, 7)]:
        m = oracle.exact_measures(sizes[p], sizes[q], inter[p, q])
        ham = np.sum(dense[p] != dense[q])
        js = np.sum(np.minimum(dense[p], dense[q])) / np.sum(np.maximum(dense[p], dense[q]))
        cos = ip[p, q] / np.linalg.norm(dense[p]) / np.linalg.norm(dense[q])
        np.testing.assert_allclose(m, [ip[p, q], ham, js, cos], rtol=1e-12)


def test_sketch_intersections_against_packed_words():
    """<a_s, b_s> by merging image sets equals the popcount of the AND of the
    packed words computed here with Python integers."""
    c = datagen.small_corpus(n=60, d=3000, seed=13)
    N = 256
    pi = datagen.random_map(c.d, N, 99)
    S = oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)
    W = oracle.pack(S, N)
    X = oracle.intersections(S, S)
    for p in range(0, 60, 7):
        for q in range(0, 60, 5):
            pc = sum(bin(int(x) & int(y)).count("1") for x, y in zip(W[p], W[q]))
            assert X[p, q] == pc


@pytest.mark.parametrize("measure", [0, 1, 2, 3])
def test_topk_against_python_sort(measure):
    c = datagen.small_corpus(n=120, d=2000, seed=14)
    N = 128
    pi = datagen.random_map(c.d, N, 5)
    S = oracle.sketch_sets(c.indptr, c.indices, c.d, pi, N)
    Q = oracle.Sets(S.vals, S.start[:10], S.length[:10])
    k = 17
    idx, sc = oracle.topk(Q, S, N, measure, k)
    X = oracle.intersections(Q, S)
    for p in range(Q.n):
        scores = [float(oracle.score_f32(Q.length[p], S.length[q], X[p, q], N, measure)) for q in range(S.n)]
        sign = 1 if measure == 1 else -1
        order = sorted(range(S.n), key=lambda q: (sign * scores[q], q))[:k]
        assert list(idx[p]) == order
        assert np.array_equal(sc[p], np.asarray([scores[q] for q in order], np.float32))


# --- Theorem 1 / Lemma 5 (weak) ---------------------------------------------------

def test_theorem1_ip_accuracy_weak():
    """At N = psi sqrt(psi/2 ln(2/delta)), |IP - n_ab| < 14 sqrt(psi/2 ln(2/delta))
    holds with probability at least 1 - 3 delta."""
    rng = np.random.default_rng(21)
    psi, delta = 40, 0.1
    P = math.sqrt(psi / 2 * math.log(2 / delta))
    N = int(math.ceil(psi * P / 64) * 64)  # rounded up to whole words
    d = 2000
    fails = 0
    trials = 300
    for _ in range(trials):
        a = rng.choice(d, psi, replace=False)
        b = np.concatenate([a[:15], rng.choice(np.setdiff1d(np.arange(d), a), psi - 15, replace=False)])
        pi = rng.integers(0, N, d).astype(np.int32)
        ip, ix = _rows_csr([a, b], d)
        S = oracle.sketch_sets(ip, ix, d, pi, N)
        x = oracle.intersections(S, S)
        e = oracle.estimate(S.length[0], S.length[1], x[0, 1], N)
        fails += abs(e[0] - 15) >= 14 * P
    assert fails / trials <= 3 * delta
