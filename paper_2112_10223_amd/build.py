"""Build of the gfx950 SpKAdd shared library (libspkadd.so) with hipcc.

Every HIP source is compiled for gfx950 only.  Packed FP32 instructions are
disabled, and the library is linked next to this file, where the Python binding
loads it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(HERE, "libspkadd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["plan_kernels.hip", "hash_kernels.hip", "wave_kernels.hip", "batch_kernels.hip", "batch_fused.hip", "bitmap_wg.hip", "unsorted_kernels.hip", "ordered.hip", "wave_fused.hip", "baselines.hip", "spkadd.cpp", "noalloc.cpp", "batch.cpp", "server.cpp",
           "autotune.cpp"]

COMMON_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build_library(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libspkadd.so.  Always rebuilds."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    return LIB_PATH


EXAMPLE_SRC = os.path.join(ROOT, "examples", "c_api.cpp")
EXAMPLE_BIN = os.path.join(ROOT, "examples", "c_api")


def build_example(verbose: bool = False) -> str:
    """Compile the C ABI example (a host program, no PyTorch) against libspkadd.so."""
    cmd = [HIPCC, *COMMON_FLAGS, EXAMPLE_SRC, "-L", HERE, "-lspkadd",
           "-Wl,-rpath,$ORIGIN/../paper_2112_10223_amd", "-o", EXAMPLE_BIN]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"example build failed:\n{res.stderr}")
    if verbose:
        print("built", EXAMPLE_BIN)
    return EXAMPLE_BIN


if __name__ == "__main__":
    build_library(verbose=True)
    build_example(verbose=True)
