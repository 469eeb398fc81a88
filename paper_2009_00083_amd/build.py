"""Build the gfx950 shared library libpcrit.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpcrit.so")
SOURCES = ["csrc/classify.hip", "csrc/api.cpp", "csrc/link_table.cpp",
           "csrc/metrics.cpp", "csrc/noalloc.hip", "csrc/classify_quad.hip",
           "csrc/learned.hip", "csrc/order.hip", "csrc/lts.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Wno-unused-result", "-Wno-unused-value",
         # keep the compiler from forming packed fp32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # f32 subnormals are kept, not flushed: the sign of a difference of
         # two subnormal samples then carries their order exactly
         "-fno-gpu-flush-denormals-to-zero"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *[os.path.join(HERE, s) for s in SOURCES]]
    res = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
