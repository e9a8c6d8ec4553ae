"""Compile the HIP sources into ``libecg.so`` (gfx950) next to this file.

Every source is compiled for gfx950 only, with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).  Objects are built in
parallel and linked into one shared library exporting the C ABI of
``include/ecg.h``.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libecg.so")
EXAMPLE = os.path.join(HERE, "examples", "poisson_solve")
SOURCES = ["ecg_kernels.hip", "ecg_api.hip", "ecg_nn.hip", "ecg_band.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{proc.stdout}\n{proc.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libecg.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed:\n{proc.stdout}\n{proc.stderr}")
    os.replace(tmp, LIB)
    # a C++ program that uses the library through include/ecg.h only (no Python)
    ex_src = os.path.join(HERE, "examples", "poisson_solve.cpp")
    if os.path.exists(ex_src):
        cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-I", os.path.join(ROOT, "include"), ex_src, "-L", HERE,
               "-lecg", f"-Wl,-rpath,{HERE}", "-o", EXAMPLE]
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError(f"example build failed:\n{proc.stdout}\n{proc.stderr}")
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
