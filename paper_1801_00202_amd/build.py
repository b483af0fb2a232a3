"""Build libmce.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libmce.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("kernels.hip", "runtime.hip")]
HEADERS = [os.path.join(PKG, "csrc", "mce_internal.h"), os.path.join(ROOT, "include", "mce.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed fp32 instructions in any device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # branches that all lanes take alike stay plain scalar branches (the
    # search loop has no lane-dependent branch; structurizing it would add
    # exec-mask bookkeeping to every child)
    "-mllvm", "-structurizecfg-skip-uniform-regions",
    "-Wall", "-Wno-unused-command-line-argument",
]


def build(force: bool = True) -> str:
    """Compile libmce.so (always, unless force is False and it is up to date)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
