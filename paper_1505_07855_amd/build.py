"""Build libbwfm.so in-tree: the host index builder with g++, the HIP kernels
and C ABI with hipcc for gfx950, linked into one shared library."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbwfm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             # no packed fp32 instructions in the device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-pthread"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = []
    o = os.path.join(OUT, "index_host.o")
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "index_host.cpp"), "-o", o])
    objs.append(o)
    for src in ("bwfm.hip", "index_gpu.hip", "rescue.hip", "mapq.hip", "server.cpp"):
        o = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
