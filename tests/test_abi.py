"""The C ABI: the library loads, exports every function include/binsketch.h
declares, and rejects bad arguments on the host before any launch (these
calls return before touching a device, so they run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "binsketch.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1910_04658_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1910_04658_amd import build
        build.build()
    return binding.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bs_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["bs_sketch", "bs_and_popcount", "bs_estimate", "bs_estimate_workspace_size", "bs_topk",
              "bs_topk_workspace_size", "bs_words", "bs_status_string", "bs_version"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), "libbinsketch.so does not export %s" % n


def test_words_and_status(lib):
    assert lib.bs_words(1024) == 16
    assert lib.bs_words(64) == 1
    assert lib.bs_words(65536) == 1024
    for bad in [0, 32, 100, 65600, -64]:
        assert lib.bs_words(bad) == 0
    assert lib.bs_status_string(0) == b"ok"
    assert lib.bs_version() >= 10000


P = ctypes.c_void_p
FAKE = P(0x1000)  # never dereferenced: every call below fails host-side validation


def test_sketch_rejects_bad_arguments(lib):
    s = lib.bs_sketch
    assert s(None, FAKE, 1, 1, FAKE, 10, 64, FAKE, None, None, None, 0, None) == 1
    assert s(FAKE, None, 1, 5, FAKE, 10, 64, FAKE, None, None, None, 0, None) == 1
    assert s(FAKE, FAKE, 1, 1, None, 10, 64, FAKE, None, None, None, 0, None) == 1
    assert s(FAKE, FAKE, 1, 1, FAKE, 10, 64, None, None, None, None, 0, None) == 1
    assert s(FAKE, FAKE, -1, 1, FAKE, 10, 64, FAKE, None, None, None, 0, None) == 2
    assert s(FAKE, FAKE, 1, -1, FAKE, 10, 64, FAKE, None, None, None, 0, None) == 2
    assert s(FAKE, FAKE, 1, 2 ** 31, FAKE, 10, 64, FAKE, None, None, None, 0, None) == 2
    assert s(FAKE, FAKE, 1, 1, FAKE, 0, 64, FAKE, None, None, None, 0, None) == 2
    for N in [0, 63, 100, 65536 + 64]:
        assert s(FAKE, FAKE, 1, 1, FAKE, 10, N, FAKE, None, None, None, 0, None) == 2


def test_prepared_map_rejects_bad_arguments(lib):
    from paper_1910_04658_amd.binding import SketchPart
    need = lib.bs_sketch_workspace_size(10, 64)
    assert need > 0
    p = lib.bs_sketch_prepare_map
    assert p(None, 10, 64, None, FAKE, need, None) == 1
    assert p(FAKE, 0, 64, None, FAKE, need, None) == 2
    assert p(FAKE, 10, 96, None, FAKE, need, None) == 2
    assert p(FAKE, 10, 64, None, None, need, None) == 3
    assert p(FAKE, 10, 64, None, FAKE, need - 1, None) == 3
    assert p(FAKE, 10, 64, None, P(0x1001), need, None) == 3
    good = SketchPart(FAKE, FAKE, 1, 1, FAKE, None)
    arr = (SketchPart * 1)(good)
    s = lib.bs_sketch_parts_prepared
    assert s(arr, 1, FAKE, 10, 64, None, need, None, None) == 3
    assert s(arr, 1, FAKE, 10, 64, FAKE, need - 1, None, None) == 3
    assert s(arr, 1, FAKE, 10, 100, FAKE, need, None, None) == 2
    assert s(arr, 0, FAKE, 10, 64, FAKE, need, None, None) == 2
    assert s(arr, 1, None, 10, 64, FAKE, need, None, None) == 1


def test_pairs_reject_bad_arguments(lib):
    assert lib.bs_and_popcount(None, 1, FAKE, 1, 64, FAKE, None) == 1
    assert lib.bs_and_popcount(FAKE, -1, FAKE, 1, 64, FAKE, None) == 2
    assert lib.bs_and_popcount(FAKE, 1, FAKE, 1, 96, FAKE, None) == 2
    assert lib.bs_and_popcount(FAKE, 2 ** 40, FAKE, 2 ** 40, 64, FAKE, None) == 2
    # estimate: no output requested, bad width, missing or short workspace
    assert lib.bs_estimate(FAKE, None, 1, FAKE, None, 1, 64, None, None, None, None, FAKE, 1 << 20, None) == 1
    assert lib.bs_estimate(FAKE, None, 1, FAKE, None, 1, 65, FAKE, None, None, None, FAKE, 1 << 20, None) == 2
    need = lib.bs_estimate_workspace_size(1, 1, 64)
    assert need > 0
    assert lib.bs_estimate(FAKE, None, 1, FAKE, None, 1, 64, FAKE, None, None, None, None, need, None) == 3
    assert lib.bs_estimate(FAKE, None, 1, FAKE, None, 1, 64, FAKE, None, None, None, FAKE, need - 1, None) == 3
    assert lib.bs_estimate(FAKE, None, 1, FAKE, None, 1, 64, FAKE, None, None, None, P(0x1001), need, None) == 3


def test_estimate_scores_rejects_bad_arguments(lib):
    f = lib.bs_estimate_scores
    need = lib.bs_estimate_workspace_size(1, 1, 64)
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 4, FAKE, 1, FAKE, need, None) == 2   # measure
    assert f(FAKE, None, 1, FAKE, None, 1, 64, -1, FAKE, 0, FAKE, need, None) == 2
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 2, FAKE, 2, FAKE, need, None) == 2   # dtype
    assert f(FAKE, None, 1, FAKE, None, 1, 96, 2, FAKE, 1, FAKE, need, None) == 2   # width
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 2, None, 1, FAKE, need, None) == 1   # no output
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 2, None, 0, FAKE, need, None) == 1
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 2, FAKE, 1, None, need, None) == 3   # workspace
    assert f(FAKE, None, 1, FAKE, None, 1, 64, 2, FAKE, 0, FAKE, need - 1, None) == 3


def test_estimate_noalloc_rejects_on_the_host(lib):
    """bs_estimate_noalloc checks its arguments as bs_estimate does, and a call
    whose row popcounts would not fit the fixed scratch (after the T table)
    returns BS_ERR_SCRATCH before any launch. At N = 64 the table takes 768
    bytes, so 1,048,384 computed popcounts fill the 4 MiB exactly and one
    more row does not fit."""
    f = lib.bs_estimate_noalloc
    assert f(FAKE, None, 1, FAKE, None, 1, 64, None, None, None, None, None) == 1    # no output
    assert f(None, None, 1, FAKE, None, 1, 64, FAKE, None, None, None, None) == 1
    assert f(FAKE, None, 1, FAKE, None, 1, 65, FAKE, None, None, None, None) == 2    # bad width
    assert f(FAKE, None, -1, FAKE, None, 1, 64, FAKE, None, None, None, None) == 2
    assert f(FAKE, None, 1_048_385, FAKE, FAKE, 1, 64, FAKE, None, None, None, None) == 6
    assert f(FAKE, FAKE, 1, FAKE, None, 1_048_385, 64, FAKE, None, None, None, None) == 6
    assert f(FAKE, None, 1_000_000, FAKE, None, 1, 65536, FAKE, None, None, None, None) == 6
    assert f(FAKE, None, 2 ** 50, FAKE, FAKE, 1, 64, FAKE, None, None, None, None) == 6
    assert lib.bs_status_string(6).startswith(b"the call needs more than the fixed no-allocation scratch")


def test_topk_rejects_bad_arguments(lib):
    t = lib.bs_topk
    need = lib.bs_topk_workspace_size(10, 100, 256, 5)
    assert need > 0
    assert t(None, None, 10, FAKE, None, 100, 256, 2, 5, FAKE, None, FAKE, need, None) == 1
    assert t(FAKE, None, 10, FAKE, None, 100, 256, 2, 5, None, None, FAKE, need, None) == 1
    assert t(FAKE, None, 10, FAKE, None, 100, 256, 2, 0, FAKE, None, FAKE, need, None) == 2     # k = 0
    assert t(FAKE, None, 10, FAKE, None, 100, 256, 2, 101, FAKE, None, FAKE, need, None) == 2   # k > nC
    assert t(FAKE, None, 10, FAKE, None, 5000, 256, 2, 1025, FAKE, None, FAKE, need, None) == 2  # k > max
    assert t(FAKE, None, 10, FAKE, None, 100, 256, 4, 5, FAKE, None, FAKE, need, None) == 2     # measure
    assert t(FAKE, None, 10, FAKE, None, 0, 256, 2, 5, FAKE, None, FAKE, need, None) == 2       # empty corpus
    assert t(FAKE, None, 10, FAKE, None, 100, 256, 2, 5, FAKE, None, FAKE, need - 1, None) == 3
    assert lib.bs_topk_workspace_size(10, 100, 256, 101) == 0
    assert lib.bs_topk_workspace_size(10, 100, 100, 5) == 0


def test_topk_plans_for_every_width_and_batch_size(lib):
    """The host plan (scan mode, slab geometry, workspace layout) for every
    width, empty and ragged batches and small and large corpora, with the
    matrix-core scan on and off: a positive size, the same whatever the
    query count for the per-corpus parts, and no host fault."""
    from paper_1910_04658_amd.binding import BatchItem
    widths = [64, 256, 320, 512, 1024, 4096, 8192, 16384, 32768, 65536]
    for on in (1, 0):
        lib.bs_debug_set_topk_mma(on)
        try:
            for N in widths:
                for nQ in (0, 1, 65, 1000):
                    for nC in (1, 100, 5000, 100_000):
                        k = min(10, nC)
                        assert lib.bs_topk_workspace_size(nQ, nC, N, k) > 0, (on, N, nQ, nC)
            # a batch large enough that the matrix-core scan would run one
            # slab per query group: the plan splits the corpus into slabs of
            # at most 2^26 rows (survivor entries keep a row's offset in
            # its slab in 26 bits)
            for N in (256, 1024):
                assert lib.bs_topk_workspace_size(400_000, 1 << 27, N, 10) > 0, (on, N)
        finally:
            lib.bs_debug_set_topk_mma(1)
    for N in widths:
        for nq in (0, 70):
            it = _batch_item(N=N, n_queries=nq, q_nnz=0 if nq == 0 else 50)
            assert lib.bs_batch_workspace_size((BatchItem * 1)(it), 1) > 0, (N, nq)


def _batch_item(**kw):
    from paper_1910_04658_amd.binding import BatchItem
    it = BatchItem()
    it.indptr = it.indices = it.q_indptr = it.q_indices = it.pi = 0x1000
    it.sketches = it.popcounts = it.q_sketches = it.q_popcounts = it.out_idx = it.out_score = 0x1000
    it.n_rows, it.nnz, it.n_queries, it.q_nnz, it.d, it.N, it.k = 100, 500, 10, 50, 1000, 256, 10
    for k, v in kw.items():
        setattr(it, k, v)
    return it


def test_batch_rejects_bad_arguments(lib):
    from paper_1910_04658_amd.binding import BatchItem
    good = _batch_item()
    arr = (BatchItem * 1)(good)
    assert lib.bs_batch_workspace_size(arr, 1) > 0
    assert lib.bs_batch_workspace_size(arr, 0) == 0
    for bad in [dict(N=100), dict(k=101), dict(k=0), dict(n_rows=0), dict(d=0), dict(nnz=-1), dict(n_queries=-1),
                dict(N=131072)]:
        assert lib.bs_batch_workspace_size((BatchItem * 1)(_batch_item(**bad)), 1) == 0, bad
    h = P()
    c = lib.bs_batch_create
    assert c(arr, 1, 2, None, 0, None, 0, None, None) == 1          # no handle out-pointer
    assert c(arr, 0, 2, None, 0, FAKE, 1 << 30, None, ctypes.byref(h)) == 2
    assert c(arr, 1, 7, None, 0, FAKE, 1 << 30, None, ctypes.byref(h)) == 2
    assert c((BatchItem * 1)(_batch_item(pi=0)), 1, 2, None, 0, FAKE, 1 << 30, None, ctypes.byref(h)) == 1
    assert c((BatchItem * 1)(_batch_item(out_idx=0)), 1, 2, None, 0, FAKE, 1 << 30, None, ctypes.byref(h)) == 1
    # no queries: the query pointers may be NULL
    assert lib.bs_batch_workspace_size((BatchItem * 1)(_batch_item(n_queries=0, q_nnz=0, q_indptr=0, q_indices=0,
                                                                   q_sketches=0, out_idx=0)), 1) > 0
    assert c(arr, 1, 2, None, 0, None, 0, None, ctypes.byref(h)) == 3   # no workspace
    assert c(arr, 1, 2, None, 0, FAKE, 16, None, ctypes.byref(h)) == 3  # too small
    assert lib.bs_batch_run(None, None) == 1
    assert lib.bs_batch_run_eager(None, None) == 1
    assert lib.bs_batch_autotune(None, 1, None) == 1
    assert lib.bs_batch_shapes(None, None, 0) == 0
    assert lib.bs_batch_graph_nodes(None) == 0
    lib.bs_batch_destroy(None)


def test_topk_sample_size(lib):
    """Rows the sample pass scores exactly: the whole corpus while it has at
    most 2,048 rows, then 2,048 up to nC / 256, growing as nC / 256 up to
    15,360 rows."""
    f = lib.bs_topk_sample_size
    assert f(0) == 0 and f(1) == 1 and f(2048) == 2048
    assert f(2049) == 2048 and f(100_000) == 2048
    assert f(600_000) == 600_000 // 256
    assert f(15360 * 256) == 15360 and f(10**9) == 15360


def test_sketch_parts_rejects_bad_arguments(lib):
    from paper_1910_04658_amd.binding import SketchPart
    s = lib.bs_sketch_parts
    good = SketchPart(FAKE, FAKE, 1, 1, FAKE, None)
    arr = (SketchPart * 5)(good, good, good, good, good)
    assert s(arr, 0, FAKE, 10, 64, None, None, 0, None) == 2  # no parts
    assert s(arr, 5, FAKE, 10, 64, None, None, 0, None) == 2  # more than BS_SKETCH_MAX_PARTS
    assert s(arr, 2, FAKE, 10, 100, None, None, 0, None) == 2  # bad width
    assert s(arr, 2, FAKE, 0, 64, None, None, 0, None) == 2    # bad d
    assert s(None, 2, FAKE, 10, 64, None, None, 0, None) == 1  # no parts array
    assert s(arr, 2, None, 10, 64, None, None, 0, None) == 1   # no map
    bad = (SketchPart * 2)(good, SketchPart(FAKE, FAKE, -1, 1, FAKE, None))
    assert s(bad, 2, FAKE, 10, 64, None, None, 0, None) == 2
    bad = (SketchPart * 2)(good, SketchPart(FAKE, FAKE, 1, 2 ** 31, FAKE, None))
    assert s(bad, 2, FAKE, 10, 64, None, None, 0, None) == 2
    bad = (SketchPart * 2)(good, SketchPart(FAKE, None, 1, 5, FAKE, None))
    assert s(bad, 2, FAKE, 10, 64, None, None, 0, None) == 1
    bad = (SketchPart * 2)(SketchPart(FAKE, FAKE, 3, 1, None, None), good)
    assert s(bad, 2, FAKE, 10, 64, None, None, 0, None) == 1
