"""Build the gfx950 shared libraries in-tree with hipcc.

``libcavi.so``        the CAVI library (include/cavi.h) and the linear-mixing VB (include/lmvb.h)
``libcavi_synth.so``  the on-device input generator (synth.py's definition)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]

LIBS = {
    "libcavi.so": ["cavi_kernels.hip", "estep_tiled.hip", "update.hip", "warmstart.hip", "lmvb.hip", "lmem.hip", "gibbs.hip", "cavi_api.cpp",
                   "warmstart_api.cpp"],
    "libcavi_synth.so": ["synth.hip"],
}


def _build_one(name: str, srcs, verbose: bool) -> str:
    out = os.path.join(HERE, name)
    tmp = out + ".tmp"
    cmd = [HIPCC, *COMMON, *[os.path.join(CSRC, s) for s in srcs], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(verbose: bool = True, only=None):
    built = []
    for name, srcs in LIBS.items():
        if only and name not in only:
            continue
        if not all(os.path.exists(os.path.join(CSRC, s)) for s in srcs):
            continue
        built.append(_build_one(name, srcs, verbose))
    return built


if __name__ == "__main__":
    for p in build(only=sys.argv[1:] or None):
        print(p)
