"""Compile libugp (the HIP library behind include/ugp.h) for gfx950, in-tree.

Usage: python -m paper_2406_09733_amd.build      (or build() from Python)

Produces paper_2406_09733_amd/libugp.so.  Each .hip source is compiled to an
object with hipcc and the objects are linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libugp.so")
OBJ = os.path.join(HERE, "_objs")
SOURCES = ["api.hip", "build.hip", "trace.hip", "render.hip", "nrc.hip", "diff.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
         # packed FP32 instructions stay off (hipcc forms them from scalar code)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-value", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(_filter(r.stderr))
    return obj


def _filter(text: str) -> str:
    # the host pass does not know the packed-fp32 feature; that note is harmless
    keep = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l]
    return ("\n".join(keep) + "\n") if any(s.strip() for s in keep) else ""


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(5, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
