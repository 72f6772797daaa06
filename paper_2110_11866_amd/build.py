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
DEVICE_SOURCES = ["scan_dispatch.hip", "direct_conv.hip", "multiply.hip", "image2d.hip", "tree.hip", "boundary.hip", "noalloc.hip"]
# scan kernel instantiation sets: scan_inst.hip once per (terms K, samples per thread R)
TERMS = range(1, 13)
TILES = (4, 8, 16, 32)
INSTANCES = [("scan_inst.hip", k, r) for k in TERMS for r in TILES]


# headers only the host sources include (a change to them leaves the device objects alone)
HOST_HEADERS = ("plan_internal.h",)


def _newest_header(host: bool) -> float:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)
            if f.endswith(".h") and (host or f not in HOST_HEADERS)]
    if host:
        hdrs.append(os.path.join(HERE, "..", "include", "morlet.h"))
    return max(os.path.getmtime(h) for h in hdrs)


# Development builds may restrict the scan kernels to some terms K (MK_DEV_TERMS="5,6"): the
# other (K, R) pairs compile as stubs without kernels. The entry build ignores it.
def _dev_terms():
    v = os.environ.get("MK_DEV_TERMS", "")
    return {int(t) for t in v.split(",") if t.strip()} if v else None


def _compile(item, incremental: bool = False, dev_terms=None) -> str:
    if isinstance(item, tuple):
        src, k, r = item
        stub = dev_terms is not None and k not in dev_terms
        obj = os.path.join(BUILD, "scan_k%d_r%d%s.o" % (k, r, "_stub" if stub else ""))
        defs = ["-DMK_K=%d" % k, "-DMK_R=%d" % r] + (["-DMK_STUB"] if stub else [])
    else:
        src, obj, defs = item, os.path.join(BUILD, os.path.splitext(item)[0] + ".o"), []
    path = os.path.join(CSRC, src)
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(path) and t > _newest_header(src.endswith(".cpp")):
            return obj
    if src.endswith(".hip"):
        cmd = [HIPCC, "-c", *COMMON, *DEVICE_FLAGS, *defs, "-x", "hip", path, "-o", obj]
    else:
        cmd = [HIPCC, "-c", *COMMON, *DEVICE_FLAGS, path, "-o", obj]   # host code, same target
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link libmorlet.so; returns its path. incremental=True keeps
    objects newer than their source and every header, and honours MK_DEV_TERMS (development
    rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    dev = _dev_terms() if incremental else None
    # the largest instantiation sets first, so the long compiles start early
    srcs = sorted(INSTANCES, key=lambda t: (-t[1], -t[2])) + DEVICE_SOURCES + HOST_SOURCES
    with ThreadPoolExecutor(max_workers=int(os.environ.get("MAX_JOBS", "8"))) as ex:
        objs = list(ex.map(lambda it: _compile(it, incremental, dev), srcs))
    tmp = OUT + ".tmp"
    subprocess.run([HIPCC, "-shared", "-fPIC", *DEVICE_FLAGS, *objs, "-o", tmp], check=True)
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
