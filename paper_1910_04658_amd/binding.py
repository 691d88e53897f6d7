"""Thin ctypes binding of libbinsketch.so (the C ABI in include/binsketch.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library. Tensors must live on the current CUDA/HIP device;
calls are enqueued on torch's current stream and return before completion,
like the C functions. Sketches are carried in int64 tensors (bit-identical to
the library's uint64 words).

If the shared library is missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbinsketch.so")

BS_OK, BS_ERR_NULL, BS_ERR_ARG, BS_ERR_WORKSPACE, BS_ERR_HIP, BS_ERR_DEVICE, BS_ERR_SCRATCH = range(7)
BS_IP, BS_HAMMING, BS_JACCARD, BS_COSINE = range(4)
FLAG_INDPTR, FLAG_INDEX, FLAG_MAP = 1, 2, 4
NOALLOC_SCRATCH_BYTES = 4 << 20  # BS_NOALLOC_SCRATCH_BYTES
MEASURES = {"ip": BS_IP, "ham": BS_HAMMING, "hamming": BS_HAMMING, "js": BS_JACCARD,
            "jaccard": BS_JACCARD, "cos": BS_COSINE, "cosine": BS_COSINE}

_lock = threading.Lock()
_lib = None


class SketchPart(ctypes.Structure):
    """bs_sketch_part (field order and types as in binsketch.h)."""
    _fields_ = [("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("sketches", ctypes.c_void_p), ("popcounts", ctypes.c_void_p)]


class BatchItem(ctypes.Structure):
    """bs_batch_item (field order and types as in binsketch.h)."""
    _fields_ = [("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("q_indptr", ctypes.c_void_p), ("q_indices", ctypes.c_void_p),
                ("n_queries", ctypes.c_int64), ("q_nnz", ctypes.c_int64),
                ("pi", ctypes.c_void_p), ("d", ctypes.c_int64),
                ("N", ctypes.c_int32), ("k", ctypes.c_int32),
                ("sketches", ctypes.c_void_p), ("popcounts", ctypes.c_void_p),
                ("q_sketches", ctypes.c_void_p), ("q_popcounts", ctypes.c_void_p),
                ("out_idx", ctypes.c_void_p), ("out_score", ctypes.c_void_p)]


class BatchShape(ctypes.Structure):
    """bs_batch_shape."""
    _fields_ = [("N", ctypes.c_int32), ("qpl", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class BinSketchError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, status_string(status), status))


def load():
    """Load libbinsketch.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libbinsketch.so is not built: run __graft_entry__.build() "
                                   "or python paper_1910_04658_amd/build.py")
            L = ctypes.CDLL(LIB_PATH)
            p, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
            L.bs_version.restype = ctypes.c_int
            L.bs_status_string.argtypes = [ctypes.c_int]
            L.bs_status_string.restype = ctypes.c_char_p
            L.bs_words.argtypes = [i32]
            L.bs_words.restype = i32
            L.bs_sketch.argtypes = [p, p, i64, i64, p, i64, i32, p, p, p, p, sz, p]
            L.bs_sketch_parts.argtypes = [ctypes.POINTER(SketchPart), i32, p, i64, i32, p, p, sz, p]
            L.bs_sketch_parts.restype = ctypes.c_int
            L.bs_sketch_prepare_map.argtypes = [p, i64, i32, p, p, sz, p]
            L.bs_sketch_prepare_map.restype = ctypes.c_int
            L.bs_sketch_parts_prepared.argtypes = [ctypes.POINTER(SketchPart), i32, p, i64, i32, p, sz, p, p]
            L.bs_sketch_parts_prepared.restype = ctypes.c_int
            L.bs_sketch_workspace_size.argtypes = [i64, i32]
            L.bs_sketch_workspace_size.restype = sz
            L.bs_sketch.restype = ctypes.c_int
            L.bs_and_popcount.argtypes = [p, i64, p, i64, i32, p, p]
            L.bs_and_popcount.restype = ctypes.c_int
            L.bs_estimate_workspace_size.argtypes = [i64, i64, i32]
            L.bs_estimate_workspace_size.restype = sz
            L.bs_estimate.argtypes = [p, p, i64, p, p, i64, i32, p, p, p, p, p, sz, p]
            L.bs_estimate.restype = ctypes.c_int
            L.bs_estimate_scores.argtypes = [p, p, i64, p, p, i64, i32, i32, p, i32, p, sz, p]
            L.bs_estimate_scores.restype = ctypes.c_int
            L.bs_estimate_noalloc.argtypes = [p, p, i64, p, p, i64, i32, p, p, p, p, p]
            L.bs_estimate_noalloc.restype = ctypes.c_int
            L.bs_topk_workspace_size.argtypes = [i64, i64, i32, i32]
            L.bs_topk_workspace_size.restype = sz
            L.bs_topk_sample_size.argtypes = [i64]
            L.bs_topk_sample_size.restype = i64
            L.bs_topk.argtypes = [p, p, i64, p, p, i64, i32, i32, i32, p, p, p, sz, p]
            L.bs_topk.restype = ctypes.c_int
            L.bs_timing_enable.argtypes = [ctypes.c_int]
            L.bs_timing_enable.restype = ctypes.c_int
            L.bs_timing_collect.restype = ctypes.c_int
            L.bs_timing_reset.restype = None
            L.bs_timing_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
            L.bs_timing_get.restype = ctypes.c_int
            L.bs_pair_popcount.argtypes = [p, i64, p, p, i64, p, i64, i32, p, p, p]
            L.bs_pair_popcount.restype = ctypes.c_int
            L.bs_mlp_param_count.restype = i32
            L.bs_mlp_workspace_size.argtypes = [i64, i32]
            L.bs_mlp_workspace_size.restype = sz
            L.bs_mlp_forward.argtypes = [p, p, p, p, i64, i32, p, p, sz, p]
            L.bs_mlp_forward.restype = ctypes.c_int
            L.bs_mlp_grad.argtypes = [p, p, p, p, p, i64, i32, p, p, p, sz, p]
            L.bs_mlp_grad.restype = ctypes.c_int
            L.bs_mlp_train_step.argtypes = [p, p, p, p, i64, ctypes.c_float, p, p, p, p, i64, i32, p, p, sz, p]
            L.bs_mlp_train_step.restype = ctypes.c_int
            L.bs_mlp_to_bf16.argtypes = [p, p, p]
            L.bs_mlp_to_bf16.restype = ctypes.c_int
            L.bs_debug_set_topk_limits.argtypes = [i64, i64]
            L.bs_debug_set_topk_limits.restype = ctypes.c_int
            L.bs_debug_set_topk_tau_rank.argtypes = [i64]
            L.bs_debug_set_topk_tau_rank.restype = ctypes.c_int
            L.bs_debug_set_topk_mma.argtypes = [i32]
            L.bs_debug_set_topk_mma.restype = ctypes.c_int
            BI, BSh = ctypes.POINTER(BatchItem), ctypes.POINTER(BatchShape)
            L.bs_batch_workspace_size.argtypes = [BI, i32]
            L.bs_batch_workspace_size.restype = sz
            L.bs_batch_create.argtypes = [BI, i32, i32, BSh, i32, p, sz, p, ctypes.POINTER(p)]
            L.bs_batch_create.restype = ctypes.c_int
            L.bs_batch_autotune.argtypes = [p, i32, p]
            L.bs_batch_autotune.restype = ctypes.c_int
            L.bs_batch_run.argtypes = [p, p]
            L.bs_batch_run.restype = ctypes.c_int
            L.bs_batch_run_eager.argtypes = [p, p]
            L.bs_batch_run_eager.restype = ctypes.c_int
            L.bs_batch_shapes.argtypes = [p, BSh, i32]
            L.bs_batch_shapes.restype = i32
            L.bs_batch_graph_nodes.argtypes = [p]
            L.bs_batch_graph_nodes.restype = i32
            L.bs_batch_destroy.argtypes = [p]
            L.bs_batch_destroy.restype = None
            _lib = L
    return _lib


def status_string(status: int) -> str:
    return load().bs_status_string(int(status)).decode()


def _check(status: int, where: str):
    if status != BS_OK:
        raise BinSketchError(status, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, name: str, dtype, ndim=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if ndim is not None and t.dim() != ndim:
        raise ValueError("%s must have %d dims" % (name, ndim))
    return t


def words(N: int) -> int:
    return int(load().bs_words(int(N)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


def sketch_workspace_size(d: int, N: int) -> int:
    return int(load().bs_sketch_workspace_size(int(d), int(N)))


def sketch(indptr: torch.Tensor, indices: torch.Tensor, pi: torch.Tensor, N: int,
           out: torch.Tensor | None = None, popcounts: bool | torch.Tensor = True,
           err_flag: torch.Tensor | None = None, workspace: torch.Tensor | None | bool = True):
    """bs_sketch: (sketches int64[n][N/64], popcounts int32[n] or None).
    workspace: a device buffer of sketch_workspace_size(d, N) bytes, True to
    allocate one, or None/False for the global-gather path."""
    _need(indptr, "indptr", torch.int32, 1)
    _need(indices, "indices", torch.int32, 1)
    _need(pi, "pi", torch.int32, 1)
    n = indptr.numel() - 1
    if n < 0:
        raise ValueError("indptr must hold n_rows + 1 entries")
    W = words(N)
    if W == 0:
        raise ValueError("invalid sketch width N=%d" % N)
    dev = indptr.device
    if out is None:
        out = torch.empty((n, W), dtype=torch.int64, device=dev)
    else:
        _need(out, "out", torch.int64, 2)
        if tuple(out.shape) != (n, W):
            raise ValueError("out must be [n_rows][N/64]")
    pop = None
    if isinstance(popcounts, torch.Tensor):
        pop = _need(popcounts, "popcounts", torch.int32, 1)
        if pop.numel() != n:
            raise ValueError("popcounts must have n_rows entries")
    elif popcounts:
        pop = torch.empty(n, dtype=torch.int32, device=dev)
    if err_flag is not None:
        _need(err_flag, "err_flag", torch.int32)
    if workspace is True:
        need = sketch_workspace_size(max(pi.numel(), 1), N)
        workspace = _workspace(need, dev) if need else None
    elif workspace is False:
        workspace = None
    wsn = workspace.numel() if workspace is not None else 0
    st = load().bs_sketch(_ptr(indptr), _ptr(indices if indices.numel() else None), n, indices.numel(),
                          _ptr(pi), pi.numel(), int(N), _ptr(out), _ptr(pop), _ptr(err_flag),
                          _ptr(workspace), wsn, _stream())
    _check(st, "bs_sketch")
    return out, pop


MAX_PARTS = 4  # BS_SKETCH_MAX_PARTS


def prepare_map(pi: torch.Tensor, N: int, err_flag: torch.Tensor | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """bs_sketch_prepare_map: pi bit-packed once, for sketch_parts(prepared=...)."""
    _need(pi, "pi", torch.int32, 1)
    need = sketch_workspace_size(max(pi.numel(), 1), N)
    if need == 0:
        raise ValueError("invalid sketch width N=%d" % N)
    if out is None:
        out = _workspace(need, pi.device)
    if err_flag is not None:
        _need(err_flag, "err_flag", torch.int32)
    st = load().bs_sketch_prepare_map(_ptr(pi), pi.numel(), int(N), _ptr(err_flag), _ptr(out), out.numel(),
                                      _stream())
    _check(st, "bs_sketch_prepare_map")
    return out


def sketch_parts(parts, pi: torch.Tensor, N: int, outs=None, popcounts=None,
                 err_flag: torch.Tensor | None = None, workspace: torch.Tensor | None | bool = True,
                 prepared: torch.Tensor | None = None):
    """bs_sketch_parts: the (indptr, indices) CSR matrices of `parts` (at most
    four) sketched with one map in one launch. outs / popcounts: optional
    lists of preallocated outputs (a None popcounts entry skips that part's
    counts). prepared: a map packed by prepare_map(pi, N), used instead of
    packing pi on this call (bs_sketch_parts_prepared). Returns
    [(sketches, popcounts), ...], each as sketch() would."""
    if not 1 <= len(parts) <= MAX_PARTS:
        raise ValueError("1 to %d parts" % MAX_PARTS)
    _need(pi, "pi", torch.int32, 1)
    W = words(N)
    if W == 0:
        raise ValueError("invalid sketch width N=%d" % N)
    arr = (SketchPart * len(parts))()
    res = []
    for i, (indptr, indices) in enumerate(parts):
        _need(indptr, "indptr", torch.int32, 1)
        _need(indices, "indices", torch.int32, 1)
        n = indptr.numel() - 1
        if n < 0:
            raise ValueError("indptr must hold n_rows + 1 entries")
        out = outs[i] if outs is not None else torch.empty((n, W), dtype=torch.int64, device=indptr.device)
        _need(out, "out", torch.int64, 2)
        if tuple(out.shape) != (n, W):
            raise ValueError("out must be [n_rows][N/64]")
        if popcounts is None:
            pop = torch.empty(n, dtype=torch.int32, device=indptr.device)
        else:
            pop = popcounts[i]
            if pop is not None:
                _need(pop, "popcounts", torch.int32, 1)
                if pop.numel() != n:
                    raise ValueError("popcounts must have n_rows entries")
        arr[i] = SketchPart(_ptr(indptr), _ptr(indices if indices.numel() else None), n, indices.numel(),
                            _ptr(out), _ptr(pop))
        res.append((out, pop))
    if err_flag is not None:
        _need(err_flag, "err_flag", torch.int32)
    if workspace is True:
        need = sketch_workspace_size(max(pi.numel(), 1), N)
        workspace = _workspace(need, pi.device) if need else None
    elif workspace is False:
        workspace = None
    wsn = workspace.numel() if workspace is not None else 0
    if prepared is not None:
        _need(prepared, "prepared map", torch.uint8, 1)
        st = load().bs_sketch_parts_prepared(arr, len(parts), _ptr(pi), pi.numel(), int(N), _ptr(prepared),
                                             prepared.numel(), _ptr(err_flag), _stream())
        _check(st, "bs_sketch_parts_prepared")
    else:
        st = load().bs_sketch_parts(arr, len(parts), _ptr(pi), pi.numel(), int(N), _ptr(err_flag),
                                    _ptr(workspace), wsn, _stream())
        _check(st, "bs_sketch_parts")
    return res


def and_popcount(A: torch.Tensor, B: torch.Tensor, N: int, out: torch.Tensor | None = None):
    """bs_and_popcount: int32[nA][nB] of |A_p AND B_q|."""
    W = words(N)
    _need(A, "A", torch.int64, 2)
    _need(B, "B", torch.int64, 2)
    if A.shape[1] != W or B.shape[1] != W:
        raise ValueError("sketch rows must hold N/64 words")
    if out is None:
        out = torch.empty((A.shape[0], B.shape[0]), dtype=torch.int32, device=A.device)
    else:
        _need(out, "out", torch.int32, 2)
    st = load().bs_and_popcount(_ptr(A), A.shape[0], _ptr(B), B.shape[0], int(N), _ptr(out), _stream())
    _check(st, "bs_and_popcount")
    return out


def _measure(measure) -> int:
    return MEASURES[measure] if isinstance(measure, str) else int(measure)


def _opt_pop(t, n, name):
    if t is None:
        return None
    _need(t, name, torch.int32, 1)
    if t.numel() != n:
        raise ValueError("%s must have one entry per row" % name)
    return t


def estimate(A: torch.Tensor, B: torch.Tensor, N: int, measures=("ip", "ham", "js", "cos"),
             workspace: torch.Tensor | None = None, popA: torch.Tensor | None = None,
             popB: torch.Tensor | None = None):
    """bs_estimate: dict measure -> float64[nA][nB]."""
    W = words(N)
    _need(A, "A", torch.int64, 2)
    _need(B, "B", torch.int64, 2)
    popA = _opt_pop(popA, A.shape[0], "popA")
    popB = _opt_pop(popB, B.shape[0], "popB")
    if A.shape[1] != W or B.shape[1] != W:
        raise ValueError("sketch rows must hold N/64 words")
    nA, nB = A.shape[0], B.shape[0]
    outs = {}
    for m in measures:
        key = {"ip": "ip", "ham": "ham", "hamming": "ham", "js": "js", "jaccard": "js",
               "cos": "cos", "cosine": "cos"}[m]
        outs[key] = torch.empty((nA, nB), dtype=torch.float64, device=A.device)
    L = load()
    need = L.bs_estimate_workspace_size(nA, nB, int(N))
    if workspace is None:
        workspace = _workspace(need, A.device)
    st = L.bs_estimate(_ptr(A), _ptr(popA), nA, _ptr(B), _ptr(popB), nB, int(N), _ptr(outs.get("ip")),
                       _ptr(outs.get("ham")),
                       _ptr(outs.get("js")), _ptr(outs.get("cos")), _ptr(workspace), workspace.numel(),
                       _stream())
    _check(st, "bs_estimate")
    return outs


def estimate_scores(A: torch.Tensor, B: torch.Tensor, N: int, measure, dtype=torch.float32,
                    workspace: torch.Tensor | None = None, popA: torch.Tensor | None = None,
                    popB: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """bs_estimate_scores: one measure's [nA][nB] scores, float32 (the values
    bs_topk ranks by) or float64 (bs_estimate's plane)."""
    W = words(N)
    _need(A, "A", torch.int64, 2)
    _need(B, "B", torch.int64, 2)
    popA = _opt_pop(popA, A.shape[0], "popA")
    popB = _opt_pop(popB, B.shape[0], "popB")
    if A.shape[1] != W or B.shape[1] != W:
        raise ValueError("sketch rows must hold N/64 words")
    if dtype not in (torch.float32, torch.float64):
        raise TypeError("dtype must be float32 or float64")
    nA, nB = A.shape[0], B.shape[0]
    if out is None:
        out = torch.empty((nA, nB), dtype=dtype, device=A.device)
    _need(out, "out", dtype, 2)
    if tuple(out.shape) != (nA, nB):
        raise ValueError("out must be [nA][nB]")
    L = load()
    if workspace is None:
        workspace = _workspace(L.bs_estimate_workspace_size(nA, nB, int(N)), A.device)
    st = L.bs_estimate_scores(_ptr(A), _ptr(popA), nA, _ptr(B), _ptr(popB), nB, int(N), _measure(measure),
                              _ptr(out), 1 if dtype == torch.float32 else 0, _ptr(workspace), workspace.numel(),
                              _stream())
    _check(st, "bs_estimate_scores")
    return out


def estimate_noalloc(A: torch.Tensor, B: torch.Tensor, N: int, measures=("ip", "ham", "js", "cos"),
                     popA: torch.Tensor | None = None, popB: torch.Tensor | None = None, outs=None):
    """bs_estimate_noalloc: bs_estimate on the library's fixed scratch (no
    workspace). `outs` (dict measure -> float64[nA][nB]) may be given, e.g.
    preallocated outside a graph capture; missing ones are allocated here."""
    W = words(N)
    _need(A, "A", torch.int64, 2)
    _need(B, "B", torch.int64, 2)
    popA = _opt_pop(popA, A.shape[0], "popA")
    popB = _opt_pop(popB, B.shape[0], "popB")
    if A.shape[1] != W or B.shape[1] != W:
        raise ValueError("sketch rows must hold N/64 words")
    nA, nB = A.shape[0], B.shape[0]
    outs = dict(outs or {})
    for m in measures:
        key = {"ip": "ip", "ham": "ham", "hamming": "ham", "js": "js", "jaccard": "js",
               "cos": "cos", "cosine": "cos"}[m]
        if key not in outs:
            outs[key] = torch.empty((nA, nB), dtype=torch.float64, device=A.device)
    for t in outs.values():
        _need(t, "output", torch.float64, 2)
        if tuple(t.shape) != (nA, nB):
            raise ValueError("outputs must be [nA][nB]")
    L = load()
    st = L.bs_estimate_noalloc(_ptr(A), _ptr(popA), nA, _ptr(B), _ptr(popB), nB, int(N), _ptr(outs.get("ip")),
                               _ptr(outs.get("ham")), _ptr(outs.get("js")), _ptr(outs.get("cos")), _stream())
    _check(st, "bs_estimate_noalloc")
    return outs


def topk_workspace_size(nQ: int, nC: int, N: int, k: int) -> int:
    return int(load().bs_topk_workspace_size(int(nQ), int(nC), int(N), int(k)))


def topk_sample_size(nC: int) -> int:
    """Corpus rows bs_topk scores exactly in its sample pass."""
    return int(load().bs_topk_sample_size(int(nC)))


def topk(Q: torch.Tensor, C: torch.Tensor, N: int, measure, k: int, scores: bool = True,
         workspace: torch.Tensor | None = None, out_idx: torch.Tensor | None = None,
         out_score: torch.Tensor | None = None, popQ: torch.Tensor | None = None,
         popC: torch.Tensor | None = None):
    """bs_topk: (idx int32[nQ][k], score float32[nQ][k] or None)."""
    m = MEASURES[measure] if isinstance(measure, str) else int(measure)
    W = words(N)
    _need(Q, "Q", torch.int64, 2)
    _need(C, "C", torch.int64, 2)
    popQ = _opt_pop(popQ, Q.shape[0], "popQ")
    popC = _opt_pop(popC, C.shape[0], "popC")
    if Q.shape[1] != W or C.shape[1] != W:
        raise ValueError("sketch rows must hold N/64 words")
    nQ, nC = Q.shape[0], C.shape[0]
    if out_idx is None:
        out_idx = torch.empty((nQ, k), dtype=torch.int32, device=Q.device)
    if out_score is None and scores:
        out_score = torch.empty((nQ, k), dtype=torch.float32, device=Q.device)
    L = load()
    need = L.bs_topk_workspace_size(nQ, nC, int(N), int(k))
    if need == 0:
        raise ValueError("invalid top-k arguments (nC=%d, N=%d, k=%d)" % (nC, N, k))
    if workspace is None:
        workspace = _workspace(need, Q.device)
    st = L.bs_topk(_ptr(Q), _ptr(popQ), nQ, _ptr(C), _ptr(popC), nC, int(N), m, int(k), _ptr(out_idx),
                   _ptr(out_score),
                   _ptr(workspace), workspace.numel(), _stream())
    _check(st, "bs_topk")
    return out_idx, out_score


def debug_set_topk_limits(slab_capacity: int = -1, lds_keys: int = -1):
    """Test hook: shrink the top-k candidate slots per slab / the LDS key
    buffer of the select (-1 = automatic)."""
    load().bs_debug_set_topk_limits(int(slab_capacity), int(lds_keys))


def debug_set_topk_tau_rank(rank: int = -1):
    """Test hook: take the filter threshold as the rank-th best sample score
    (below the automatic rank; -1 = automatic)."""
    load().bs_debug_set_topk_tau_rank(int(rank))


def debug_set_topk_mma(on: bool = True):
    """Test hook: False forms the scan's pair counts on the vector ALU even
    where the matrix-core scan applies (True = automatic)."""
    load().bs_debug_set_topk_mma(1 if on else 0)


def timing_enable(on: bool = True):
    load().bs_timing_enable(1 if on else 0)


def timing_reset():
    load().bs_timing_reset()


def timing_collect() -> int:
    return int(load().bs_timing_collect())


def timing_get(name: str):
    """(total milliseconds, launch count) recorded for a kernel name."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    load().bs_timing_get(name.encode(), ctypes.byref(ms), ctypes.byref(n))
    return ms.value, n.value


def pair_popcount(A: torch.Tensor, ia: torch.Tensor, B: torch.Tensor, ib: torch.Tensor, N: int,
                  out: torch.Tensor | None = None, err_flag: torch.Tensor | None = None):
    """bs_pair_popcount: int32[n] of |A[ia[i]] AND B[ib[i]]|."""
    _need(A, "A", torch.int64, 2)
    _need(B, "B", torch.int64, 2)
    _need(ia, "ia", torch.int32, 1)
    _need(ib, "ib", torch.int32, 1)
    if ia.numel() != ib.numel():
        raise ValueError("ia and ib must have the same length")
    if out is None:
        out = torch.empty(ia.numel(), dtype=torch.int32, device=A.device)
    st = load().bs_pair_popcount(_ptr(A), A.shape[0], _ptr(ia), _ptr(B), B.shape[0], _ptr(ib), ia.numel(),
                                 int(N), _ptr(out), _ptr(err_flag), _stream())
    _check(st, "bs_pair_popcount")
    return out


def mlp_param_count() -> int:
    return int(load().bs_mlp_param_count())


def mlp_workspace(n: int, N: int, device) -> torch.Tensor:
    return _workspace(load().bs_mlp_workspace_size(int(n), int(N)), device)


def _counts(xa, xb, xab):
    for t, nm in ((xa, "xa"), (xb, "xb"), (xab, "xab")):
        _need(t, nm, torch.int32, 1)
    if not (xa.numel() == xb.numel() == xab.numel()):
        raise ValueError("xa, xb, xab must have the same length")
    return xa.numel()


def mlp_forward(w_bf16: torch.Tensor, xa, xb, xab, N: int, out=None, workspace=None):
    """bs_mlp_forward: learned Jaccard estimates, float32[n]."""
    _need(w_bf16, "w", torch.int16, 1)
    n = _counts(xa, xb, xab)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xa.device)
    if workspace is None:
        workspace = mlp_workspace(n, N, xa.device)
    st = load().bs_mlp_forward(_ptr(w_bf16), _ptr(xa), _ptr(xb), _ptr(xab), n, int(N), _ptr(out),
                               _ptr(workspace), workspace.numel(), _stream())
    _check(st, "bs_mlp_forward")
    return out


def mlp_grad(w_bf16: torch.Tensor, xa, xb, xab, label: torch.Tensor, N: int, workspace=None):
    """bs_mlp_grad: (grad float32[4545], loss float32[1])."""
    _need(w_bf16, "w", torch.int16, 1)
    _need(label, "label", torch.float32, 1)
    n = _counts(xa, xb, xab)
    grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=xa.device)
    loss = torch.empty(1, dtype=torch.float32, device=xa.device)
    if workspace is None:
        workspace = mlp_workspace(n, N, xa.device)
    st = load().bs_mlp_grad(_ptr(w_bf16), _ptr(xa), _ptr(xb), _ptr(xab), _ptr(label), n, int(N), _ptr(grad),
                            _ptr(loss), _ptr(workspace), workspace.numel(), _stream())
    _check(st, "bs_mlp_grad")
    return grad, loss


def mlp_train_step(master, w_bf16, adam_m, adam_v, step: int, lr: float, xa, xb, xab, label, N: int,
                   loss=None, workspace=None):
    """bs_mlp_train_step (in place on master, w_bf16, adam_m, adam_v)."""
    n = _counts(xa, xb, xab)
    if workspace is None:
        workspace = mlp_workspace(n, N, xa.device)
    st = load().bs_mlp_train_step(_ptr(master), _ptr(w_bf16), _ptr(adam_m), _ptr(adam_v), int(step), float(lr),
                                  _ptr(xa), _ptr(xb), _ptr(xab), _ptr(label), n, int(N), _ptr(loss),
                                  _ptr(workspace), workspace.numel(), _stream())
    _check(st, "bs_mlp_train_step")


def mlp_to_bf16(master: torch.Tensor, w_bf16: torch.Tensor):
    st = load().bs_mlp_to_bf16(_ptr(master), _ptr(w_bf16), _stream())
    _check(st, "bs_mlp_to_bf16")


class Batch:
    """A batch of independent problems (bs_batch_*): each problem is a dict
    with device tensors `indptr`, `indices` (corpus CSR, int32), `q_indptr`,
    `q_indices` (query CSR), `pi` (int32[d]) and ints `d`, `N`, `k`. Output
    tensors are allocated here, per problem: sketches, popcounts, q_sketches,
    q_popcounts, idx, score. `shapes`: tuned shapes as returned by shapes()."""

    def __init__(self, problems: list, measure="js", shapes=None, device=None):
        L = load()
        m = MEASURES[measure] if isinstance(measure, str) else int(measure)
        dev = device if device is not None else problems[0]["indptr"].device
        self.problems = problems
        self.out = []
        arr = (BatchItem * len(problems))()
        for i, pb in enumerate(problems):
            for name in ("indptr", "indices", "q_indptr", "q_indices", "pi"):
                _need(pb[name], name, torch.int32, 1)
            N, k = int(pb["N"]), int(pb["k"])
            W = N // 64
            n, nq = pb["indptr"].numel() - 1, pb["q_indptr"].numel() - 1
            o = {"sketches": torch.empty((n, W), dtype=torch.int64, device=dev),
                 "popcounts": torch.empty(n, dtype=torch.int32, device=dev),
                 "q_sketches": torch.empty((max(nq, 0), W), dtype=torch.int64, device=dev),
                 "q_popcounts": torch.empty(max(nq, 0), dtype=torch.int32, device=dev),
                 "idx": torch.empty((max(nq, 0), k), dtype=torch.int32, device=dev),
                 "score": torch.empty((max(nq, 0), k), dtype=torch.float32, device=dev)}
            self.out.append(o)
            it = arr[i]
            it.indptr, it.indices = pb["indptr"].data_ptr(), pb["indices"].data_ptr()
            it.n_rows, it.nnz = n, pb["indices"].numel()
            it.q_indptr, it.q_indices = pb["q_indptr"].data_ptr(), pb["q_indices"].data_ptr()
            it.n_queries, it.q_nnz = nq, pb["q_indices"].numel()
            it.pi, it.d, it.N, it.k = pb["pi"].data_ptr(), int(pb["d"]), N, k
            it.sketches, it.popcounts = o["sketches"].data_ptr(), o["popcounts"].data_ptr()
            it.q_sketches, it.q_popcounts = o["q_sketches"].data_ptr(), o["q_popcounts"].data_ptr()
            it.out_idx, it.out_score = o["idx"].data_ptr(), o["score"].data_ptr()
        self._items = arr
        nbytes = L.bs_batch_workspace_size(arr, len(problems))
        if nbytes == 0:
            raise BinSketchError(BS_ERR_ARG, "bs_batch_workspace_size")
        self.workspace = _workspace(nbytes, dev)
        self.err = torch.zeros(len(problems), dtype=torch.int32, device=dev)
        sh = None
        if shapes:
            sh = (BatchShape * len(shapes))()
            for j, x in enumerate(shapes):
                sh[j].N, sh[j].qpl, sh[j].waves, sh[j].ms = int(x["N"]), int(x["qpl"]), int(x["waves"]), float(x.get("ms", -1))
        h = ctypes.c_void_p()
        torch.cuda.synchronize(dev)
        _check(L.bs_batch_create(arr, len(problems), m, sh, len(shapes) if shapes else 0, _ptr(self.workspace),
                                 self.workspace.numel(), _ptr(self.err), ctypes.byref(h)), "bs_batch_create")
        self._h = h

    def autotune(self, reps: int = 3):
        _check(load().bs_batch_autotune(self._h, int(reps), _stream()), "bs_batch_autotune")

    def run(self):
        _check(load().bs_batch_run(self._h, _stream()), "bs_batch_run")

    def run_eager(self):
        _check(load().bs_batch_run_eager(self._h, _stream()), "bs_batch_run_eager")

    def shapes(self) -> list:
        L = load()
        n = L.bs_batch_shapes(self._h, None, 0)
        arr = (BatchShape * max(n, 1))()
        L.bs_batch_shapes(self._h, arr, n)
        return [{"N": arr[j].N, "qpl": arr[j].qpl, "waves": arr[j].waves, "ms": arr[j].ms} for j in range(n)]

    def graph_nodes(self) -> int:
        return int(load().bs_batch_graph_nodes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load().bs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
