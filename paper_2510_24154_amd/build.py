"""Build the engine's shared library for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libepidmc.so")
SOURCES = ["epidmc.cpp", "tables.cpp", "kernels.hip", "unet.hip", "microbench.hip"]
# FP32 division and square root at the hardware's 1-2.5 ulp instead of correctly rounded
# sequences, and FP32 denormals flushed: no FP32 quantity of the transport comes near the
# denormal range, and the tallies and positions that need more than FP32 are FP64
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-o", tmp,
                        "-x", "hip", *[os.path.join(CSRC, s) for s in SOURCES]],
                       capture_output=not verbose, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + (r.stderr or "")[-6000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
