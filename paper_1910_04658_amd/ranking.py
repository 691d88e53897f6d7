"""Threshold-retrieval quality of the sketch estimates (Section 4.2, Experiment 2).

For every query, O holds the corpus rows whose exact similarity reaches a
threshold and O' those whose estimated similarity (bs_estimate on the
sketches) does. O' is scored against O by accuracy |O∩O'|/|O∪O'|, precision
|O∩O'|/|O'|, recall |O∩O'|/|O| and F1 = 2PR/(P+R), with the sets holding
(query, row) pairs pooled over all queries. Empty denominators: an empty union
scores accuracy 1, an empty O' precision 1, an empty O recall 1, and F1 is 0
when P + R is 0.

Thresholds: the paper's set for Jaccard and cosine; for the inner product the
same fractions of the largest exact inner product among the pairs.
"""
from __future__ import annotations

import numpy as np

THRESHOLDS = (0.95, 0.9, 0.85, 0.8, 0.6, 0.5, 0.2, 0.1)


def set_metrics(truth: np.ndarray, found: np.ndarray) -> dict:
    """Metrics of the pair mask `found` (O') against the pair mask `truth` (O)."""
    truth = np.asarray(truth, bool)
    found = np.asarray(found, bool)
    inter = int(np.count_nonzero(truth & found))
    union = int(np.count_nonzero(truth | found))
    nt = int(np.count_nonzero(truth))
    nf = int(np.count_nonzero(found))
    acc = inter / union if union else 1.0
    prec = inter / nf if nf else 1.0
    rec = inter / nt if nt else 1.0
    f1 = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
    return {"accuracy": acc, "precision": prec, "recall": rec, "f1": f1, "truth": nt, "found": nf}


def threshold_metrics(est: np.ndarray, exact: np.ndarray, thresholds=THRESHOLDS) -> dict:
    """{threshold: set_metrics(exact >= t, est >= t)} for similarities."""
    est = np.asarray(est)
    exact = np.asarray(exact)
    return {float(t): set_metrics(exact >= t, est >= t) for t in thresholds}


def ip_thresholds(exact_ip: np.ndarray, fractions=THRESHOLDS) -> list:
    """Inner-product thresholds: fractions of the largest exact inner product."""
    m = float(np.max(exact_ip)) if np.size(exact_ip) else 0.0
    return [f * m for f in fractions]
