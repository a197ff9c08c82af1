"""Build libepic.so for gfx950 with hipcc (in-tree, no JIT cache).

Usage: ``python -m paper_2609_03027_amd.build`` or ``build_library()``.
Every HIP source is compiled with packed-FP32 instruction selection turned
off; each translation unit is compiled in parallel and then linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libepic.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["abi.hip", "plan.hip", "fused.hip", "banded.hip", "staged.hip", "readout.hip", "dftgemm.hip",
           "fixed.hip", "sep.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


def _compile(src: str, obj: str, extra) -> tuple[str, int, str]:
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    return src, r.returncode, msg


def build_library(verbose: bool = False, extra=()) -> str:
    """Compile every source and link ``libepic.so``; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = []
        for src in SOURCES:
            obj = os.path.join(BUILD, src.replace(".hip", ".o"))
            objs.append(obj)
            futs.append(ex.submit(_compile, src, obj, list(extra)))
        errors = []
        for f in futs:
            src, rc, msg = f.result()
            if msg.strip() and (verbose or rc):
                print(f"[{src}]\n{msg}", file=sys.stderr)
            if rc:
                errors.append(src)
    if errors:
        raise RuntimeError(f"hipcc failed for {errors}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
