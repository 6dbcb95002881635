"""Build libqed.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2008_10468_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqed.so")
PEAKS_LIB = os.path.join(HERE, "libqed_peaks.so")
ARCH = os.environ.get("QED_OFFLOAD_ARCH", "gfx950")

SOURCES = ["qed_kernels.hip", "qed_train.hip", "qed_grid.hip", "qed_capi.hip"]
PEAKS_SOURCES = ["qed_peaks.hip"]   # measurement microbenchmarks, a library of their own

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-fvisibility=hidden",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused within one expression only, never across
    # statements, so that a function inlined into different kernels rounds the
    # same way in each (the schedulers must give bit-identical results)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _link(cc, sources, lib, verbose):
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in sources:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [cc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    cc = hipcc()
    _link(cc, PEAKS_SOURCES, PEAKS_LIB, verbose)
    return _link(cc, SOURCES, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
