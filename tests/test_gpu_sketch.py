"""bs_sketch against the CPU oracle: sketch words and popcounts bit-exact."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import to_dev, words_np

pytestmark = pytest.mark.gpu


def run_sketch(csr, pi, N, dev, err=False, workspace=True):
    """workspace=True: map packed into a workspace and kept in LDS (when it
    fits); workspace=False: every map entry gathered from global memory."""
    import torch
    from paper_1910_04658_amd import binding as bs
    flag = torch.zeros(1, dtype=torch.int32, device=dev) if err else None
    w, p = bs.sketch(to_dev(csr.indptr, dev), to_dev(csr.indices, dev), to_dev(pi, dev), N, err_flag=flag,
                     workspace=workspace)
    torch.cuda.synchronize()
    return words_np(w), p.cpu().numpy(), (int(flag.item()) if err else None)


def check(csr, pi, N, dev):
    ow, op = oracle.sketch(csr.indptr, csr.indices, csr.d, pi, N)
    for ws in (True, False):
        gw, gp, flag = run_sketch(csr, pi, N, dev, err=True, workspace=ws)
        assert flag == 0
        assert np.array_equal(gw, ow), "sketch words differ (workspace=%s)" % ws
        assert np.array_equal(gp, op), "popcounts differ (workspace=%s)" % ws


def test_small_corpus_N1024(dev):
    """1,000 vectors, d = 10,000, Zipf lengths in [5, 500], N = 1024."""
    c = datagen.small_corpus()
    check(c, datagen.random_map(c.d, 1024, datagen.SEED_PI), 1024, dev)


@pytest.mark.parametrize("N", [64, 128, 192, 256, 320, 512, 1024, 2048, 4096, 8192, 16384, 65536])
def test_widths(N, dev):
    c = datagen.small_corpus(n=300, d=20000, seed=N)
    check(c, datagen.random_map(c.d, N, N + 1), N, dev)


def test_adversarial_rows(dev):
    """Empty rows, single-element rows, rows far longer than one chunk or one
    window, duplicates and unsorted indices, and a stretch of empty rows."""
    rng = np.random.default_rng(3)
    d = 50000
    rows = [[], [7], [], [], list(rng.integers(0, d, 5000)), [3, 3, 3, 1, 1]]
    rows += [[] for _ in range(70)]
    rows += [list(rng.integers(0, d, int(m))) for m in rng.integers(0, 40, 200)]
    rows += [list(rng.permutation(d)[:20000])]
    rows += [[d - 1, 0]] * 3 + [[]]
    c = datagen.from_rows(rows, d)
    for N in [64, 1024, 8192]:
        check(c, datagen.random_map(d, N, 5), N, dev)


def test_all_indices_to_one_bucket(dev):
    c = datagen.small_corpus(n=200, d=3000, seed=4)
    for j in [0, 63, 64, 1023]:
        pi = np.full(c.d, j, np.int32)
        check(c, pi, 1024, dev)


def test_identity_map_gives_the_vector(dev):
    d = N = 4096
    c = datagen.small_corpus(n=100, d=d, seed=8)
    gw, gp, _ = run_sketch(c, np.arange(d, dtype=np.int32), N, dev)
    for r in range(c.n):
        bits = np.zeros(N, np.uint8)
        bits[c.row(r)] = 1
        packed = np.packbits(bits, bitorder="little").view(np.uint64)
        assert np.array_equal(gw[r], packed)


def test_empty_batches(dev):
    import torch
    from paper_1910_04658_amd import binding as bs
    pi = to_dev(np.zeros(10, np.int32), dev)
    w, p = bs.sketch(to_dev(np.zeros(1, np.int32), dev), to_dev(np.zeros(0, np.int32), dev), pi, 64)
    torch.cuda.synchronize()
    assert w.shape == (0, 1) and p.shape == (0,)
    c = datagen.from_rows([[] for _ in range(100)], 10)
    gw, gp, flag = run_sketch(c, np.zeros(10, np.int32), 128, dev, err=True)
    assert flag == 0 and not gw.any() and not gp.any()


def test_deterministic_across_runs(dev):
    c = datagen.small_corpus(n=2000, d=10000, seed=9)
    pi = datagen.random_map(c.d, 512, 9)
    a = run_sketch(c, pi, 512, dev)
    b = run_sketch(c, pi, 512, dev)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_error_flags(dev):
    """Malformed content is reported through the device flag; the kernel's own
    bounds checks keep every access in bounds."""
    d, N = 100, 128
    pi = datagen.random_map(d, N, 1)
    for ws in (True, False):
        c = datagen.from_rows([[1, 2], [5, 100], [3]], d)  # index 100 >= d
        _, _, flag = run_sketch(c, pi, N, dev, err=True, workspace=ws)
        assert flag & 2
        pi_bad = pi.copy()
        pi_bad[7] = N  # map value out of range
        c = datagen.from_rows([[1, 7], [3]], d)
        _, _, flag = run_sketch(c, pi_bad, N, dev, err=True, workspace=ws)
        assert flag & 4
        c = datagen.from_rows([[1, 2], [3, 4]], d)
        c.indptr[2] = 2  # 0, 2, 2 is fine; 0, 3, 2 is not non-decreasing
        c.indptr[1] = 3
        _, _, flag = run_sketch(c, pi, N, dev, err=True, workspace=ws)
        assert flag & 1


@pytest.mark.parametrize("N", [256, 1024, 4096])
def test_full_size_corpus(N, dev):
    """100,000 vectors, d = 100,000, log-normal lengths (mean 230, sd 150):
    every sketch word and popcount against the oracle."""
    c = _big_corpus()
    check(c, datagen.random_map(c.d, N, datagen.SEED_PI + N), N, dev)


def _big_corpus():
    from conftest import shared_input
    return shared_input("corpus100k", lambda: datagen.lognormal_corpus(100_000))



@pytest.mark.parametrize("N", [256, 1024, 4096])
def test_parts_equal_single_calls(N, dev):
    """bs_sketch_parts over a corpus, its queries, an empty matrix and a
    one-row matrix (one map, one launch) writes for every part exactly what
    bs_sketch writes for it alone, with the map in LDS and gathered from
    global memory; one part is also checked against the oracle."""
    import torch
    from paper_1910_04658_amd import binding as bs
    corpus = datagen.lognormal_corpus(30000, d=40000, seed=31)
    queries = datagen.lognormal_corpus(700, d=40000, seed=32)
    tiny = datagen.lognormal_corpus(1, d=40000, seed=33)
    empty_ptr = torch.zeros(1, dtype=torch.int32, device=dev)
    empty_idx = torch.zeros(0, dtype=torch.int32, device=dev)
    pi_np = datagen.random_map(40000, N, 34)
    pi = to_dev(pi_np, dev)
    mats = [corpus, queries, None, tiny]
    parts = [(empty_ptr, empty_idx) if m is None else (to_dev(m.indptr, dev), to_dev(m.indices, dev)) for m in mats]
    for ws in (True, False):
        flag = torch.zeros(1, dtype=torch.int32, device=dev)
        res = bs.sketch_parts(parts, pi, N, err_flag=flag, workspace=ws)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        for (ip, ix), (w, p) in zip(parts, res):
            w1, p1 = bs.sketch(ip, ix, pi, N, workspace=ws)
            torch.cuda.synchronize()
            assert torch.equal(w, w1) and torch.equal(p, p1)
    ow, op = oracle.sketch(queries.indptr, queries.indices, queries.d, pi_np, N)
    assert np.array_equal(words_np(res[1][0]), ow) and np.array_equal(res[1][1].cpu().numpy(), op)


def test_parts_error_flag(dev):
    """An index outside [0, d) in one part raises the call's flag."""
    import torch
    from paper_1910_04658_amd import binding as bs
    a = datagen.lognormal_corpus(2000, d=5000, seed=35)
    b = datagen.lognormal_corpus(300, d=5000, seed=36)
    ix = b.indices.copy()
    ix[7] = 5000 + 3
    pi = to_dev(datagen.random_map(5000, 1024, 37), dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    bs.sketch_parts([(to_dev(a.indptr, dev), to_dev(a.indices, dev)), (to_dev(b.indptr, dev), to_dev(ix, dev))],
                    pi, 1024, err_flag=flag)
    torch.cuda.synchronize()
    assert int(flag.item()) & bs.FLAG_INDEX


@pytest.mark.parametrize("N", [256, 1024, 4096, 16384])
def test_prepared_map_equals_per_call_packing(N, dev):
    """A map packed once by bs_sketch_prepare_map and reused by
    bs_sketch_parts_prepared gives exactly the sketches and popcounts of
    bs_sketch_parts (which packs the map on every call), over two calls in a
    row on different inputs (d = 100,000); at N = 16384 the packed map
    (175 KB) does not fit in LDS and both take the gathered path."""
    import torch
    from paper_1910_04658_amd import binding as bs
    pi_np = datagen.random_map(100_000, N, 41)
    pi = to_dev(pi_np, dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    packed = bs.prepare_map(pi, N, err_flag=flag)
    for seed in (42, 43):
        a = datagen.lognormal_corpus(5000, d=100_000, seed=seed)
        b = datagen.lognormal_corpus(300, d=100_000, seed=seed + 100)
        parts = [(to_dev(a.indptr, dev), to_dev(a.indices, dev)), (to_dev(b.indptr, dev), to_dev(b.indices, dev))]
        got = bs.sketch_parts(parts, pi, N, err_flag=flag, prepared=packed)
        want = bs.sketch_parts(parts, pi, N, err_flag=flag)
        torch.cuda.synchronize()
        for (w, p), (w1, p1) in zip(got, want):
            assert torch.equal(w, w1) and torch.equal(p, p1)
    assert int(flag.item()) == 0
    ow, op = oracle.sketch(b.indptr, b.indices, b.d, pi_np, N)
    assert np.array_equal(words_np(got[1][0]), ow) and np.array_equal(got[1][1].cpu().numpy(), op)


def test_prepare_map_flags_bad_values(dev):
    """Map values outside [0, N) are reported when the map is prepared."""
    import torch
    from paper_1910_04658_amd import binding as bs
    pi_np = datagen.random_map(5000, 1024, 44)
    pi_np[123] = 1024
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    bs.prepare_map(to_dev(pi_np, dev), 1024, err_flag=flag)
    torch.cuda.synchronize()
    assert int(flag.item()) & bs.FLAG_MAP
