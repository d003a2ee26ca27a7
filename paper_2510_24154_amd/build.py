"""Build the engine's shared library for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libepidmc.so")
SOURCES = ["epidmc.cpp", "tables.cpp", "kernels.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
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
