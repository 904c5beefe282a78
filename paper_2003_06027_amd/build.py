"""Build libseisgrad.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2003_06027_amd.build  (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libseisgrad.so")
SOURCES = ["seisgrad.hip", "ac2.hip", "ad2.hip", "ac3.hip", "el2.hip", "util.hip", "cnn.hip", "lbfgs.hip", "sources.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (hipcc would otherwise emit them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-fvisibility=hidden",
]


def build(verbose: bool = False, extra=()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    out = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", out] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
