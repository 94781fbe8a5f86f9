"""Build libkc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1403_0734_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkc.so")
PEAKS_LIB = os.path.join(PKG, "libkc_peaks.so")
ARCH = os.environ.get("KC_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", INCLUDE, "-I", CSRC,
    # keep the compiler from emitting packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # hipcc's host pass warns that it does not know the packed-fp32 feature; drop that noise
    noise = ("packed-fp32-ops", "is not a recognized feature", "warning generated", "warnings generated")
    msg = "\n".join(line for line in r.stderr.splitlines() if line.strip() and not any(x in line for x in noise))
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(jobs: int = 8) -> str:
    """libkc.so (the counting library) and libkc_peaks.so (peak microbenchmarks)."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    peaks = os.path.join(CSRC, "peaks", "kc_peaks.hip")
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs) + 1)) as ex:
        objs = list(ex.map(_compile, srcs + [peaks]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], PEAKS_LIB)
    return LIB


if __name__ == "__main__":
    print(build())
