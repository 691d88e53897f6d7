"""Batched execution (bs_batch_*): many uneven problems (sizes, dimensions,
widths, query counts) sketched and ranked by one graph launch must give, for
every problem, exactly what bs_sketch and bs_topk give on it alone, and what
the CPU oracle gives."""
import numpy as np
import pytest

import datagen
import oracle
from helpers import assert_topk_equal, sets_rows, words_np

pytestmark = pytest.mark.gpu


def small_batch(dev):
    """Nine problems covering both scan modes (<= 64 and > 64 queries), a
    problem with no queries, one query, every batch width and a width with a
    non-power-of-two word count (N = 320)."""
    from conftest import shared_input

    def make():
        specs = datagen.batch_specs(n_problems=9, seed=4101, n_lo=300, n_hi=7000, d_lo=2000, d_hi=60000,
                                    m_lo=5.0, m_hi=150.0, widths=(128, 512, 2048, 8192, 320), q_min=3)
        specs[0].nq = 90
        specs[1].nq = 0
        specs[2].nq = 1
        specs[3].nq = 130
        specs[4].N = 320
        return specs
    specs = shared_input("batch_specs_small", make)
    return specs, datagen.device_batch(specs, dev, k=40)


def single_calls(pb, measure):
    """Each problem through bs_sketch and bs_topk alone."""
    from paper_1910_04658_amd import binding as bs
    N, k = pb["N"], pb["k"]
    C, pC = bs.sketch(pb["indptr"], pb["indices"], pb["pi"], N)
    Q, pQ = bs.sketch(pb["q_indptr"], pb["q_indices"], pb["pi"], N)
    if Q.shape[0] == 0:
        return C, pC, Q, pQ, None, None
    idx, sc = bs.topk(Q, C, N, measure, k, popQ=pQ, popC=pC)
    return C, pC, Q, pQ, idx, sc


def assert_same(batch, problems, measure):
    import torch
    torch.cuda.synchronize()
    for i, pb in enumerate(problems):
        C, pC, Q, pQ, idx, sc = single_calls(pb, measure)
        o = batch.out[i]
        assert torch.equal(o["sketches"], C), "problem %d: corpus sketches differ" % i
        assert torch.equal(o["popcounts"], pC), "problem %d: corpus popcounts differ" % i
        assert torch.equal(o["q_sketches"], Q), "problem %d: query sketches differ" % i
        assert torch.equal(o["q_popcounts"], pQ), "problem %d: query popcounts differ" % i
        if idx is not None:
            assert torch.equal(o["idx"], idx), "problem %d: top-k indices differ" % i
            assert torch.equal(o["score"].view(torch.int32), sc.view(torch.int32)), "problem %d: scores differ" % i


@pytest.mark.parametrize("measure", ["js", "ham", "cos", "ip"])
def test_batch_graph_equals_single_calls(measure, dev):
    from paper_1910_04658_amd import binding as bs
    specs, problems = small_batch(dev)
    b = bs.Batch(problems, measure)
    b.run()
    assert_same(b, problems, measure)
    assert b.graph_nodes() >= 3
    assert int(b.err.abs().sum().item()) == 0
    b.close()


def test_batch_against_oracle(dev):
    """Two problems checked against the CPU oracle (sketch bits and top-k)."""
    import torch
    from paper_1910_04658_amd import binding as bs
    specs, problems = small_batch(dev)
    b = bs.Batch(problems, "js")
    b.run()
    torch.cuda.synchronize()
    for i in (0, 5):
        pb = problems[i]
        ip, ix = pb["indptr"].cpu().numpy(), pb["indices"].cpu().numpy()
        qp, qx = pb["q_indptr"].cpu().numpy(), pb["q_indices"].cpu().numpy()
        pi = pb["pi"].cpu().numpy()
        SC = oracle.sketch_sets(ip, ix, pb["d"], pi, pb["N"])
        SQ = oracle.sketch_sets(qp, qx, pb["d"], pi, pb["N"])
        assert (words_np(b.out[i]["sketches"]) == oracle.pack(SC, pb["N"])).all()
        nq = len(qp) - 1
        sel = np.arange(0, nq, max(1, nq // 10))
        oi, osc = oracle.topk(sets_rows(SQ, sel), SC, pb["N"], oracle.JS, pb["k"])
        assert_topk_equal(b.out[i]["idx"].cpu().numpy()[sel], b.out[i]["score"].cpu().numpy()[sel], oi, osc)
    b.close()


def test_batch_graph_replays(dev):
    """Every replay recomputes everything: outputs are wiped between replays
    (eager torch work on the same stream) and must come back identical."""
    import torch
    from paper_1910_04658_amd import binding as bs
    specs, problems = small_batch(dev)
    b = bs.Batch(problems, "js")
    b.run()
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in b.out]
    for rep in range(3):
        for o in b.out:
            for v in o.values():
                v.fill_(-1)
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for i, o in enumerate(b.out):
            for key, v in o.items():
                assert torch.equal(v, ref[i][key]), "replay %d, problem %d: %s differs" % (rep, i, key)
    b.close()


def test_batch_autotune_keeps_results(dev):
    """Tuning picks a shape per width (with a measured time) and changes no
    result; a batch built from the tuned shapes gives the same results too."""
    import torch
    from paper_1910_04658_amd import binding as bs
    specs, problems = small_batch(dev)
    b = bs.Batch(problems, "cos")
    b.autotune(reps=1)
    shapes = b.shapes()
    assert sorted(s["N"] for s in shapes) == sorted({p["N"] for p in problems})
    ranked = {p["N"] for p, sp in zip(problems, specs) if sp.nq > 0}
    assert all(s["ms"] >= 0 and s["qpl"] in (1, 2, 4) and s["waves"] > 0 for s in shapes if s["N"] in ranked)
    b.run()
    assert_same(b, problems, "cos")
    b2 = bs.Batch(problems, "cos", shapes=shapes)
    b2.run_eager()
    torch.cuda.synchronize()
    for o1, o2 in zip(b.out, b2.out):
        for key in o1:
            assert torch.equal(o1[key], o2[key])
    b.close()
    b2.close()


def test_batch_error_flags_per_problem(dev):
    """A map value outside [0, N) in one problem and an index outside [0, d)
    in another raise only those problems' flags (the run clears the flags)."""
    import torch
    from paper_1910_04658_amd import binding as bs
    specs, problems = small_batch(dev)
    bad = [dict(p) for p in problems]
    pi = bad[2]["pi"].clone()
    pi[int(bad[2]["indices"][0].item())] = bad[2]["N"] + 5
    bad[2]["pi"] = pi
    ix = bad[6]["indices"].clone()
    ix[3] = bad[6]["d"] + 100
    bad[6]["indices"] = ix
    b = bs.Batch(bad, "js")
    b.err.fill_(77)
    b.run()
    torch.cuda.synchronize()
    err = b.err.cpu().numpy()
    assert err[2] & bs.FLAG_MAP and err[6] & bs.FLAG_INDEX
    assert (np.delete(err, [2, 6]) == 0).all()
    b.close()
