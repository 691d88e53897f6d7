"""BinSketch CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference for everything the GPU library
computes. Only ``tests/``, the package smoke check and the benchmark's CPU
baseline may import this package; the library never does, and the two share no
code. The arithmetic lives in ``binsketch_oracle.c`` (plain C, FP64) and in the
small pure-Python helpers below; this module compiles the C file with gcc and
calls it through ctypes.

Parity pins (what ties this oracle to the paper rather than to itself) are in
``tests/test_oracle_pins.py``; every function here is pinned there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from fractions import Fraction
from itertools import product

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "binsketch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

ERR_INDEX, ERR_MAP, ERR_INDPTR, ERR_ARG = 1, 2, 4, 8
IP, HAM, JS, COS = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (always when force, else only if missing)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            p = ctypes.c_void_p
            i64 = ctypes.c_int64
            i32 = ctypes.c_int32
            L.orc_set_threads.argtypes = [ctypes.c_int]
            L.orc_normalize.argtypes = [p, p, i64, i64, p, p]
            L.orc_sketch_sets.argtypes = [p, p, i64, i64, p, i32, p, p]
            L.orc_pack.argtypes = [p, p, p, i64, i32, p]
            L.orc_intersections.argtypes = [p, p, p, i64, p, p, p, i64, p]
            L.orc_exact_measures.argtypes = [i64, i64, i64, p]
            L.orc_exact_measures.restype = None
            L.orc_estimate_literal.argtypes = [ctypes.c_double] * 4 + [p]
            L.orc_estimate_literal.restype = None
            L.orc_estimate_canonical.argtypes = [i64, i64, i64, i64, p]
            L.orc_estimate_canonical.restype = None
            L.orc_score_f32.argtypes = [i64, i64, i64, i64, ctypes.c_int]
            L.orc_score_f32.restype = ctypes.c_float
            L.orc_estimate_pairs.argtypes = [p, i64, p, i64, p, i32, p]
            L.orc_topk.argtypes = [p, p, p, i64, p, p, p, i64, i32, ctypes.c_int, i32, p, p]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the C oracle; returns the count in use."""
    return int(lib().orc_set_threads(int(n)))


class Sets:
    """Rows as sorted distinct lists: row r is vals[start[r] : start[r] + length[r]]."""

    def __init__(self, vals, start, length):
        self.vals = np.ascontiguousarray(vals, dtype=np.int32)
        self.start = np.ascontiguousarray(start, dtype=np.int32)
        self.length = np.ascontiguousarray(length, dtype=np.int32)

    @property
    def n(self):
        return len(self.length)

    def row(self, r):
        s = int(self.start[r])
        return self.vals[s:s + int(self.length[r])]


def _csr_arrays(indptr, indices):
    return (np.ascontiguousarray(indptr, dtype=np.int32),
            np.ascontiguousarray(indices, dtype=np.int32))


def normalize(indptr, indices, d) -> Sets:
    """CSR rows -> sorted distinct index lists (binary semantics)."""
    ip, ix = _csr_arrays(indptr, indices)
    n = len(ip) - 1
    vals = np.zeros(max(len(ix), 1), np.int32)
    ln = np.zeros(n, np.int32)
    err = lib().orc_normalize(_ptr(ip), _ptr(ix), n, int(d), _ptr(vals), _ptr(ln))
    if err:
        raise ValueError("oracle: malformed input (code %d)" % err)
    return Sets(vals, ip[:-1], ln)


def sketch_sets(indptr, indices, d, pi, N) -> Sets:
    """Sketch images S_a = sorted distinct {pi[i] : i in a} (Definition BinSketch)."""
    ip, ix = _csr_arrays(indptr, indices)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    n = len(ip) - 1
    vals = np.zeros(max(len(ix), 1), np.int32)
    ln = np.zeros(n, np.int32)
    err = lib().orc_sketch_sets(_ptr(ip), _ptr(ix), n, int(d), _ptr(pi), int(N), _ptr(vals), _ptr(ln))
    if err:
        raise ValueError("oracle: malformed input (code %d)" % err)
    return Sets(vals, ip[:-1], ln)


def pack(sets: Sets, N: int) -> np.ndarray:
    """Pack sets to uint64[n][N/64], bit j -> word j//64, bit j%64."""
    out = np.zeros((sets.n, N // 64), np.uint64)
    rc = lib().orc_pack(_ptr(sets.vals), _ptr(sets.start), _ptr(sets.length), sets.n, int(N), _ptr(out))
    if rc:
        raise ValueError("oracle: bad pack arguments")
    return out


def sketch(indptr, indices, d, pi, N):
    """(packed sketches uint64[n][N/64], |a_s| int32[n])."""
    s = sketch_sets(indptr, indices, d, pi, N)
    return pack(s, N), s.length.copy()


def intersections(A: Sets, B: Sets) -> np.ndarray:
    out = np.zeros((A.n, B.n), np.int32)
    lib().orc_intersections(_ptr(A.vals), _ptr(A.start), _ptr(A.length), A.n,
                            _ptr(B.vals), _ptr(B.start), _ptr(B.length), B.n, _ptr(out))
    return out


def exact_measures(na, nb, nab) -> np.ndarray:
    out = np.zeros(4, np.float64)
    lib().orc_exact_measures(int(na), int(nb), int(nab), _ptr(out))
    return out


def estimate_literal(xa, xb, xab, N) -> np.ndarray:
    """Algorithms 1-4 as printed (Hamming with the factor 2), real inputs, FP64."""
    out = np.zeros(4, np.float64)
    lib().orc_estimate_literal(float(xa), float(xb), float(xab), float(N), _ptr(out))
    return out


def estimate(xa, xb, xab, N) -> np.ndarray:
    """Canonical FP64 estimates (IP, Ham, JS, Cos) from integer counts."""
    out = np.zeros(4, np.float64)
    lib().orc_estimate_canonical(int(xa), int(xb), int(xab), int(N), _ptr(out))
    return out


def score_f32(xa, xb, xab, N, measure) -> np.float32:
    return np.float32(lib().orc_score_f32(int(xa), int(xb), int(xab), int(N), int(measure)))


def estimate_pairs(xa, xb, xab, N) -> np.ndarray:
    """Dense canonical estimates: float64[4][nA][nB] (IP, Ham, JS, Cos)."""
    xa = np.ascontiguousarray(xa, np.int32)
    xb = np.ascontiguousarray(xb, np.int32)
    xab = np.ascontiguousarray(xab, np.int32)
    out = np.zeros((4, len(xa), len(xb)), np.float64)
    lib().orc_estimate_pairs(_ptr(xa), len(xa), _ptr(xb), len(xb), _ptr(xab), int(N), _ptr(out))
    return out


def topk(Q: Sets, C: Sets, N: int, measure: int, k: int):
    """Top-k corpus rows per query by FP32 score: (idx int32[nQ][k], score f32[nQ][k])."""
    idx = np.zeros((Q.n, k), np.int32)
    sc = np.zeros((Q.n, k), np.float32)
    rc = lib().orc_topk(_ptr(Q.vals), _ptr(Q.start), _ptr(Q.length), Q.n,
                        _ptr(C.vals), _ptr(C.start), _ptr(C.length), C.n,
                        int(N), int(measure), int(k), _ptr(idx), _ptr(sc))
    if rc:
        raise ValueError("oracle: bad top-k arguments")
    return idx, sc


# ---------------------------------------------------------------------------
# Pure-Python pieces for tiny inputs
# ---------------------------------------------------------------------------

def sketch_by_definition(a_bits, pi, N):
    """a_s[j] = OR of a[i] over i with pi(i) = j, coordinate by coordinate
    (Section 3, Definition "BinSketch"), for a dense 0/1 list a_bits."""
    out = [0] * N
    for j in range(N):
        v = 0
        for i in range(len(a_bits)):
            if pi[i] == j:
                v = v | a_bits[i]
        out[j] = v
    return out


def enumerate_expectations(d, N, a, b):
    """Exact E|a_s| and E<a_s, b_s> over all N^d maps pi (each equally likely,
    as the Definition makes pi uniform over the N^d functions), as Fractions.
    Sketches come from :func:`sketch_sets`, intersections from :func:`intersections`."""
    ia = np.asarray([0, len(a)], np.int32)
    ib = np.asarray([0, len(b)], np.int32)
    tot_a = 0
    tot_ab = 0
    count = 0
    for pi in product(range(N), repeat=d):
        pi = np.asarray(pi, np.int32)
        sa = sketch_sets(ia, np.asarray(a, np.int32), d, pi, N)
        sb = sketch_sets(ib, np.asarray(b, np.int32), d, pi, N)
        tot_a += int(sa.length[0])
        tot_ab += int(intersections(sa, sb)[0, 0])
        count += 1
    return Fraction(tot_a, count), Fraction(tot_ab, count)
