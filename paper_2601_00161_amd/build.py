"""Build the gfx950 shared library in-tree with hipcc.

``python -m paper_2601_00161_amd.build`` (or ``build()``) compiles every
source under ``csrc/`` and links ``libesp_mi355x.so`` next to this file.  It
always recompiles; nothing is cached between calls.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libesp_mi355x.so")

ARCH = "gfx950"
SOURCES = ["esp_kernels.hip", "esp_real.hip", "esp_mlp.hip", "esp_plan.cpp", "esp_noalloc.hip", "pswf.cpp"]
# compiled once per window support P, to instantiate the P-specialised kernels in parallel
PER_P = ("esp_stencil.hip", range(2, 13))
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res


def build(verbose: bool = False) -> str:
    """Compile all sources and link the library; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    hipcc = _hipcc()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = []
    for s in srcs:
        obj = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        jobs.append([hipcc, *FLAGS, *lang, "-c", os.path.join(CSRC, s), "-o", obj])
    src, ps = PER_P
    for P in ps:
        obj = os.path.join(OBJ, f"{os.path.splitext(src)[0]}_p{P}.o")
        jobs.append([hipcc, *FLAGS, f"-DESP_P={P}", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
