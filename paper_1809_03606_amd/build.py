"""Build the HIP library ``libpolarscs.so`` in-tree with hipcc for gfx950.

Run ``python -m paper_1809_03606_amd.build`` (or ``__graft_entry__.build()``).  The
library is what the Python binding loads; nothing is built at import time.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpolarscs.so")
# the LDS bandwidth microbenchmark (a measurement aid, not part of the decoder library)
LDS_PEAK_LIB = os.path.join(PKG, "libldspeak.so")
BUILD_DIR = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
SOURCES = ["polar_code.cpp", "scs_decode.hip", "fsscs_decode.hip", "scl_decode.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "-Wall",
          "-fno-fast-math", "-ffp-contract=off"]
# Device code: gfx950 only; no packed-fp32 instructions (see the design notes).  The
# decoders' control flow is wave-uniform (one frame per wavefront, every branch on scalar
# values), so LLVM's CFG structurizer is told to leave uniform regions alone: it would
# otherwise rewrite them into predicated form with extra scalar flag bookkeeping on every
# branch, and the decoders are bound by scalar instruction issue.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mllvm", "-structurizecfg-skip-uniform-regions=1"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + DEVICE
    else:
        cmd += ["-x", "c++"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES) + 1) as ex:
        objs = list(ex.map(_compile, SOURCES + ["lds_peak.hip"]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], LDS_PEAK_LIB)
    if verbose:
        print("built", LIB, LDS_PEAK_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
