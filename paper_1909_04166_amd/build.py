"""Build ``libcmlb.so`` (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(``-target-feature -packed-fp32-ops``) and with multiply-add contraction limited
to single source expressions (``-ffp-contract=on``): every kernel instantiation
(workgroup width, prefetch variant) then rounds identically, so a lattice gives
the same bits alone, in a batch or under any tile shape.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcmlb.so")
SOURCES = ["lb_kernels.hip", "lb_aux.hip", "lb_capi.hip"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=on", "-Wno-unused-command-line-argument"]
# roctx ranges around the stepping calls (marker traces)
LIBS = ["-L" + os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
        "-lrocprofiler-sdk-roctx"]


STAMP_SUFFIX = ".srchash"


def source_hash(extra: list[str] | None = None) -> str:
    """Hash of everything the library is compiled from: the HIP sources and
    headers, the public header and the compiler flags."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    for f in files + [os.path.join("..", "..", "include", "cmlb.h")]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    h.update(" ".join(FLAGS + (extra or []) + LIBS).encode())
    return h.hexdigest()[:32]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compiles the library and writes the hash of its sources beside it
    (``libcmlb.so.srchash``); the binding refuses a library whose hash does not
    match the sources in the tree."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = out or LIB
    tmp = lib + ".tmp"
    digest = source_hash(extra)
    cmd = [hipcc] + FLAGS + (extra or []) + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    with open(lib + STAMP_SUFFIX, "w") as fh:
        fh.write(digest + "\n")
    return lib


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
