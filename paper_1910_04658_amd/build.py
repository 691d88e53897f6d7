"""Builds libbinsketch.so (all HIP sources, gfx950) in the package directory."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbinsketch.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["capi.cpp", "sketch.hip", "pairs.hip", "topk.hip", "mlp.hip", "batch.hip"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    # packed FP32 VALU forms are switched off for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    srcs = []
    for s in SOURCES:
        path = os.path.join(CSRC, s)
        if s.endswith(".cpp"):
            srcs += ["-x", "hip", path]
        else:
            srcs.append(path)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + (extra or []) + ["-I", INCLUDE, "-I", CSRC] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
