"""Build the gfx950 shared libraries in-tree with hipcc.

``libcavi.so``        the CAVI library (include/cavi.h) and the paper's linear-mixing procedures
                      (include/lmvb.h, lmem.h, gibbs.h)
``libcavi_synth.so``  the on-device input generator (synth.py's definition)

Each source is compiled to an object of its own (in parallel, under ``_build/``), then the objects
are linked; no device code calls across sources.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]

LIBS = {
    "libcavi.so": ["cavi_kernels.hip", "estep_tiled.hip", "update.hip", "warmstart.hip", "lmvb.hip", "lmem.hip",
                   "gibbs.hip", "cavi_static.hip", "cavi_api.cpp", "warmstart_api.cpp"],
    "libcavi_synth.so": ["synth.hip"],
}


def _compile(src: str, csrc: str, obj_dir: str, verbose: bool) -> str:
    obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *COMMON, *lang, "-c", os.path.join(csrc, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def _build_one(name: str, srcs, verbose: bool, csrc: str, out_dir: str, obj_dir: str, jobs: int) -> str:
    os.makedirs(obj_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, csrc, obj_dir, verbose), srcs))
    out = os.path.join(out_dir, name)
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(verbose: bool = True, only=None, csrc: str = CSRC, out_dir: str = HERE, obj_dir: str = OBJ):
    jobs = max(1, min(8, os.cpu_count() or 1))
    built = []
    for name, srcs in LIBS.items():
        if only and name not in only:
            continue
        if not all(os.path.exists(os.path.join(csrc, s)) for s in srcs):
            continue
        built.append(_build_one(name, srcs, verbose, csrc, out_dir, os.path.join(obj_dir, name), jobs))
    return built


if __name__ == "__main__":
    for p in build(only=sys.argv[1:] or None):
        print(p)
