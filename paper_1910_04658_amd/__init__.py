"""BinSketch on MI355X (gfx950): sketching of sparse binary vectors and
sketch-only estimation of inner product, Hamming, Jaccard and cosine
similarity (Pratap, Bera, Revanuru, arXiv 1910.04658).

The computation lives in libbinsketch.so (HIP kernels behind the C ABI of
include/binsketch.h); ``binding`` marshals torch device tensors into it.
Importing the package does not load the library; the first call does, and
raises if it has not been built.
"""
from . import binding  # noqa: F401
from .binding import (BS_COSINE, BS_HAMMING, BS_IP, BS_JACCARD, and_popcount,  # noqa: F401
                      estimate, sketch, topk, words)

__all__ = ["binding", "sketch", "and_popcount", "estimate", "topk", "words",
           "BS_IP", "BS_HAMMING", "BS_JACCARD", "BS_COSINE"]
