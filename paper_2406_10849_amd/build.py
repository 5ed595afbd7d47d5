"""Build libgmot.so in-tree with hipcc for gfx950.

Usage: ``python -m paper_2406_10849_amd.build`` (or ``build()`` from Python).
Every build compiles from source; the library lands next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgmot.so")

SOURCES = ["gmot_kernels.hip", "gmot_round.hip", "gmot_mlp.hip", "gmot_runtime.cpp"]

# Packed FP32 instructions are switched off for every HIP object; the
# host pass reports that it does not know the feature, which is harmless.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; a ROCm toolchain is required to build libgmot")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objs = []
    tmp = LIB + ".tmp"
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    for src in srcs:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_" + os.path.splitext(src)[0] + ".o")
        cmd = [cc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip", "-c", path, "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
