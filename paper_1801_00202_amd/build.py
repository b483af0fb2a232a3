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


PROBE_LIB = os.path.join(PKG, "libmce_probe.so")
PROBE_SOURCES = [os.path.join(PKG, "csrc", "probe.hip")]
PROBE_HEADERS = [os.path.join(ROOT, "include", "mce_probe.h")]


def _compile(lib: str, sources, headers, force: bool) -> str:
    if not force and os.path.exists(lib):
        newest = max(os.path.getmtime(p) for p in sources + headers)
        if os.path.getmtime(lib) >= newest:
            return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *sources]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(force: bool = True) -> str:
    """Compile libmce.so and the peak-rate probes libmce_probe.so (always,
    unless force is False and they are up to date)."""
    _compile(PROBE_LIB, PROBE_SOURCES, PROBE_HEADERS, force)
    return _compile(LIB, SOURCES, HEADERS, force)


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
