"""Threshold-retrieval metrics (Section 4.2, Experiment 2): the oracle's
plain-set definitions pinned by hand-computed cases, and the library's
vectorised version checked against the oracle."""
import numpy as np
import pytest

from oracle import ranking as oref


def test_oracle_metrics_by_hand():
    """O = {(0,1), (0,2), (1,3)}, O' = {(0,2), (1,3), (1,4), (2,0)}:
    |O∩O'| = 2, |O∪O'| = 5, so accuracy 2/5, precision 2/4, recall 2/3 and
    F1 = 2 (1/2)(2/3) / (1/2 + 2/3) = 4/7."""
    O = {(0, 1), (0, 2), (1, 3)}
    Op = {(0, 2), (1, 3), (1, 4), (2, 0)}
    m = oref.set_metrics(O, Op)
    assert m["accuracy"] == pytest.approx(2 / 5)
    assert m["precision"] == pytest.approx(1 / 2)
    assert m["recall"] == pytest.approx(2 / 3)
    assert m["f1"] == pytest.approx(4 / 7)
    assert (m["truth"], m["found"]) == (3, 4)


def test_oracle_metrics_special_cases():
    O = {(0, 0), (1, 1)}
    assert oref.set_metrics(O, set(O)) == {"accuracy": 1.0, "precision": 1.0, "recall": 1.0, "f1": 1.0,
                                           "truth": 2, "found": 2}
    m = oref.set_metrics(O, {(2, 2)})
    assert (m["accuracy"], m["precision"], m["recall"], m["f1"]) == (0.0, 0.0, 0.0, 0.0)
    m = oref.set_metrics(set(), set())
    assert (m["accuracy"], m["precision"], m["recall"], m["f1"]) == (1.0, 1.0, 1.0, 1.0)
    m = oref.set_metrics(set(), {(0, 0)})
    assert (m["accuracy"], m["precision"], m["recall"], m["f1"]) == (0.0, 0.0, 1.0, 0.0)
    m = oref.set_metrics(O, set())
    assert (m["accuracy"], m["precision"], m["recall"], m["f1"]) == (0.0, 1.0, 0.0, 0.0)


def test_oracle_retrieved():
    s = [[0.5, 0.95, 0.1], [0.96, 0.2, 0.95]]
    assert oref.retrieved(s, 0.95) == {(0, 1), (1, 0), (1, 2)}
    assert oref.retrieved(s, 0.2, higher_is_better=False) == {(0, 2), (1, 1)}


def test_library_metrics_match_oracle():
    from paper_1910_04658_amd import ranking
    rng = np.random.default_rng(7)
    for trial in range(30):
        shape = (int(rng.integers(1, 9)), int(rng.integers(1, 9)))
        exact = rng.random(shape)
        est = exact + rng.normal(0, 0.15, shape) * (rng.random() < 0.8)
        lib = ranking.threshold_metrics(est, exact)
        for t in ranking.THRESHOLDS:
            ref = oref.set_metrics(oref.retrieved(exact.tolist(), t), oref.retrieved(est.tolist(), t))
            assert lib[t] == pytest.approx(ref)


def test_ip_thresholds():
    from paper_1910_04658_amd import ranking
    assert ranking.ip_thresholds(np.array([[3.0, 40.0], [7.0, 1.0]]), (0.5, 0.1)) == [20.0, 4.0]
    assert ranking.ip_thresholds(np.zeros((0, 0)), (0.5,)) == [0.0]
