"""Build the native libraries in-tree.

  librichtess.so  host input stage (g++, C++17)
  librich.so      device path: HIP kernels for gfx950 and the C-ABI (hipcc)

Every call compiles (no staleness shortcut): the caller decides when to build.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
TESS_SRC = os.path.join(HERE, "host", "tess.cpp")
TESS_LIB = os.path.join(HERE, "librichtess.so")
HIP_SRCS = [os.path.join(HERE, "csrc", f) for f in ("rich_kernels.hip", "rich_retess.hip")]
HIP_LIB = os.path.join(HERE, "librich.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# HIP flags: gfx950 only; packed-FP32 instructions disabled (see the
# kernels' header comment); no fast-math so that divisions and square roots
# are IEEE-correct like the oracle's.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall",
]


def _run(cmd):
    print("+", " ".join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)


def build_tess():
    tmp = TESS_LIB + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
          "-pthread", "-I", INCLUDE, TESS_SRC, "-o", tmp])
    os.replace(tmp, TESS_LIB)
    return TESS_LIB


def build_hip():
    srcs = [s for s in HIP_SRCS if os.path.exists(s)]
    if not srcs:
        return None
    tmp = HIP_LIB + ".tmp"
    _run([os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-I", INCLUDE, *srcs,
          "-o", tmp])
    os.replace(tmp, HIP_LIB)
    return HIP_LIB


def build_all():
    build_tess()
    build_hip()


if __name__ == "__main__":
    build_all()
