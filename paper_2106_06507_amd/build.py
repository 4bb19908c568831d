"""Build libbg.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Usage: python -m paper_2106_06507_amd.build   (or build_library() from Python)
Objects go to _build/ at the repository root; the shared library is written
next to this file so that it travels with the source tree.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbg.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off: the compiler must not emit v_pk_* f32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]

SOURCES = ["bg_api.cpp", "colour_matrix.cpp", "cobg_pair.hip", "cobg_adj.hip", "cdbg.hip",
           "contract.hip", "batch.hip", "rambo.hip", "comc.hip", "cdmc.hip", "util.hip",
           "noalloc.hip", "full_colour.hip", "batch_kinds_all.hip", "batch_kinds_cobg.hip",
           "batch_kinds_cdbg.hip", "hsum.hip"]


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build_library(extra_flags=(), verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra_flags)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for (o, err) in results:
            if err.strip():
                print(f"--- {os.path.basename(o)}\n{err}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    extra = sys.argv[1:]
    print(build_library(extra_flags=extra, verbose=True))
