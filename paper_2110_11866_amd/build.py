"""Build libmorlet.so (the C ABI of include/morlet.h) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmorlet.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include")]

HOST_SOURCES = ["plan.cpp", "api.cpp"]
DEVICE_SOURCES = ["scan_dispatch.hip", "direct_conv.hip"] + ["scan_k%d.hip" % k for k in range(1, 13)]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-c", *COMMON, *DEVICE_FLAGS, "-x", "hip", path, "-o", obj]
    else:
        cmd = [HIPCC, "-c", *COMMON, *DEVICE_FLAGS, path, "-o", obj]   # host code, same target
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libmorlet.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = DEVICE_SOURCES + HOST_SOURCES
    with ThreadPoolExecutor(max_workers=int(os.environ.get("MAX_JOBS", "8"))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    subprocess.run([HIPCC, "-shared", "-fPIC", *DEVICE_FLAGS, *objs, "-o", tmp], check=True)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
