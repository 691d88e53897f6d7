"""Threshold-retrieval quality — CPU oracle (TEST INFRASTRUCTURE ONLY).

The ranking experiment of Section 4.2 (Experiment 2): for every query, O is the
set of corpus points whose exact similarity reaches a threshold and O' the set
whose similarity estimated from the sketches does. The paper scores O' against
O by
  accuracy  = |O ∩ O'| / |O ∪ O'|
  precision = |O ∩ O'| / |O'|
  recall    = |O ∩ O'| / |O|
  F1        = 2 precision recall / (precision + recall).
Here the sets hold (query, point) pairs pooled over all queries. Where a
denominator is empty the paper is silent; the reading taken is that an empty
union scores accuracy 1 (nothing to find and nothing found), an empty O'
precision 1, an empty O recall 1, and F1 is 0 when precision + recall is 0.

Written with plain Python sets from those definitions; the library's
vectorised version is checked against it.
"""
from __future__ import annotations


def retrieved(scores, threshold, higher_is_better=True):
    """{(i, j) : scores[i][j] >= threshold} (<= when lower is better)."""
    out = set()
    for i, row in enumerate(scores):
        for j, v in enumerate(row):
            if (v >= threshold) if higher_is_better else (v <= threshold):
                out.add((i, j))
    return out


def set_metrics(truth: set, found: set) -> dict:
    """Accuracy, precision, recall and F1 of `found` (O') against `truth` (O)."""
    inter = len(truth & found)
    union = len(truth | found)
    acc = inter / union if union else 1.0
    prec = inter / len(found) if found else 1.0
    rec = inter / len(truth) if truth else 1.0
    f1 = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
    return {"accuracy": acc, "precision": prec, "recall": rec, "f1": f1,
            "truth": len(truth), "found": len(found)}
