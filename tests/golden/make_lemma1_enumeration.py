"""Writes lemma1_enumeration.json: exact expectations of |a_s| and <a_s, b_s>
averaged over every map pi:[d] -> [N] (Section 3, Lemma 1), computed by the
CPU oracle alone (oracle.enumerate_expectations). The test compares these
stored rationals with Lemma 1's closed forms."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CASES = [
    # (d, N, a, b)
    (5, 3, [0, 1, 2], [1, 2, 3, 4]),
    (4, 4, [0, 1], [1, 2, 3]),
    (6, 3, [0, 1, 2, 3], [2, 3, 4, 5]),
    (5, 2, [0, 1, 2, 3], [0, 4]),
    (4, 5, [0], [1, 2]),
]


def main():
    out = []
    for d, N, a, b in CASES:
        ea, eab = oracle.enumerate_expectations(d, N, a, b)
        out.append({"d": d, "N": N, "a": a, "b": b,
                    "E_pop_a": "%d/%d" % (ea.numerator, ea.denominator),
                    "E_and_ab": "%d/%d" % (eab.numerator, eab.denominator)})
    doc = {"source": "exhaustive enumeration of all N^d maps by oracle.enumerate_expectations",
           "pins": "Section 3, Lemma 1 (both parts)", "cases": out}
    with open(os.path.join(HERE, "lemma1_enumeration.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
