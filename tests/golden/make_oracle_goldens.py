"""Write the oracle reference images that the GPU parity tests at the benchmark geometry
compare with: the coupled workload's 256 x 256 x 128 phantom of 2 mm voxels, its spectrum and
4-layer EPID at the native 0.39 mm pixel pitch, under narrow open fields.

    python tests/golden/make_oracle_goldens.py [--threads N] [--only NAME]

Calls only the CPU oracle (oracle/) and the seeded input generators (synth); each file holds
the mean image (MeV per history per pixel), the variance of that mean, the history count, the
oracle seed and the SHA-256 of the oracle source it came from, which a CPU test checks
against the current source.

  oracle_narrow_field_native.npz  1 x 1 cm field, 64 x 64 image: the native-pitch z-gate
                                  (a few hundred phosphor deposits per in-field pixel)
  oracle_narrow_field_g3.npz      1.5 x 1.5 cm field, 96 x 96 image: the 2%/2 mm gamma gate on
                                  8 x 8-binned pixels (3.12 mm), sigma-bar <= 1% after binning
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

GOLDENS = {
    "oracle_narrow_field_native": {"field": 1.0, "npx": 64, "histories": 16_000_000, "seed": 1001},
    "oracle_narrow_field_g3": {"field": 1.5, "npx": 96, "histories": 120_000_000, "seed": 1002},
}


def oracle_source_sha() -> str:
    return hashlib.sha256(open(os.path.join(ROOT, "oracle", "epid_oracle.c"), "rb").read()).hexdigest()


def make(name: str, threads: int, parts: int = 40) -> str:
    import oracle
    from paper_2510_24154_amd import synth
    g = GOLDENS[name]
    cfg = synth.narrow_field(field=g["field"], npx=g["npx"])
    P = oracle.Prepared(cfg, g["seed"])
    n, m = g["histories"], g["histories"] // parts
    s = np.zeros(P.npix)
    s2 = np.zeros(P.npix)
    t0 = time.time()
    for i in range(parts):   # in parts, to report progress; the sums are the same
        first = i * m
        cnt = m if i < parts - 1 else n - first
        _, _, si, s2i, _ = oracle.run(cfg, cnt, seed=g["seed"], first=first, threads=threads, prepared=P)
        s += si
        s2 += s2i
        print(f"[{name}] {first + cnt}/{n} histories, {time.time() - t0:.0f} s", flush=True)
    mean = s / n
    var = np.maximum((s2 / n - mean * mean) / (n - 1), 0.0)
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, mean=mean.reshape(P.shape), var=var.reshape(P.shape), histories=n, seed=g["seed"],
                        field_cm=g["field"], npx=g["npx"], pitch_cm=0.039, oracle_sha=oracle_source_sha())
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=list(GOLDENS), default=None)
    a = ap.parse_args()
    for name in ([a.only] if a.only else list(GOLDENS)):
        print(make(name, a.threads), flush=True)
