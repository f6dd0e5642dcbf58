"""Builds libsgmi.so (the HIP library behind include/sg.h) for gfx950 with hipcc.

    python -m paper_1906_11195_amd.build

Every call recompiles all sources (in parallel) into
``paper_1906_11195_amd/_build/`` and links ``paper_1906_11195_amd/libsgmi.so``.
``SG_BUILD_DEFINES`` (space-separated) adds compiler definitions, e.g.
``SG_BUILD_DEFINES=-DSG_SK_PROF=1`` for the SK sweep's per-role cycle counters.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsgmi.so")
SOURCES = ["sg_host.cpp", "sg_vb.hip", "sg_vbm.hip", "sg_sk.hip", "sg_skg.hip", "sg_measure.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def _flags():
    return ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            # keep packed-FP32 instructions out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"] + os.environ.get("SG_BUILD_DEFINES", "").split()


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *_flags(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
