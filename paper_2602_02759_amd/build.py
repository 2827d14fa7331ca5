"""Build libnnef.so in-tree with hipcc for gfx950.

Every source is compiled to an object in parallel, then linked into
``paper_2602_02759_amd/libnnef.so``.  Objects go to ``_build/`` at the
repository root (not committed).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnnef.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["kernels.hip", "learned.hip", "fused16.hip", "fused16bf.hip", "fused16h.hip", "fused32.hip",
           "fused32bf.hip", "fused32h.hip", "fused64.hip", "fused64bf.hip", "fused64h.hip", "fused16b.hip",
           "fused32b.hip", "fused64b.hip", "noalloc.hip", "direct.hip", "planner.cpp", "abi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(INCLUDE, "nnef.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, defines=(), tag="", incremental=False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _newest_header():
            return obj
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], *lang, "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=(), incremental: bool = False) -> str:
    """Compile and link; ``defines`` are passed to every compile as -D options.
    ``incremental`` reuses objects newer than their source and every header."""
    os.makedirs(BUILD, exist_ok=True)
    tag = "".join("." + d.replace("=", "_") for d in defines)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines, tag, incremental), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
