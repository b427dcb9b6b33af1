"""Build libmfft.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed FP32 instructions
disabled, in parallel, then linked into paper_2602_23525_amd/libmfft.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmfft.so")

SOURCES = [
    "k_c32_k0.hip", "k_c32_k1.hip", "k_c32_k5.hip", "k_c32_k7.hip", "k_c64_k0.hip",
    "k_c64_k1.hip", "k_c64_k5.hip", "k_c64_k7.hip", "k_c32_k0_e24.hip", "k_c32_k1_e24.hip",
    "k_c64_k0_e24.hip", "k_c64_k1_e24.hip",
    "k_leaf.hip", "k_leaf_batch.hip", "kernels.hip", "problem.cpp", "plan.cpp", "tune.cpp", "api.cpp", "batch.cpp", "server.cpp",
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
         "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    path = os.path.join(SRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC, *FLAGS, *lang, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(SRC, s))]
    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-Wl,-soname,libmfft.so"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
