"""Write the oracle reference images that the GPU parity tests at the benchmark geometry
compare with: the coupled workload's 256 x 256 x 128 phantom of 2 mm voxels, its spectrum and
4-layer EPID at the native 0.39 mm pixel pitch, under narrow open fields.

    python tests/golden/make_oracle_goldens.py [--threads N] [--only NAME] [--extend]

--extend keeps an existing file made by the same oracle source with the same seed and runs only
the history ids it lacks, [stored count, target count), adding their sums to the stored ones
(the oracle's result for a history depends only on its id, so this equals one run over all ids
up to the order of the sums).
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
    "oracle_narrow_field_g3": {"field": 1.5, "npx": 96, "histories": 160_000_000, "seed": 1002},
}


def oracle_source_sha() -> str:
    return hashlib.sha256(open(os.path.join(ROOT, "oracle", "epid_oracle.c"), "rb").read()).hexdigest()


def stored_sums(path, seed):
    """(histories, sum, sum of squares) of an existing file made by the current oracle source
    with this seed, or None.  Files without stored sums get them back from the mean and the
    variance of the mean: s = n m, s2 = n (var (n - 1) + m^2)."""
    if not os.path.exists(path):
        return None
    d = np.load(path)
    if str(d["oracle_sha"]) != oracle_source_sha() or int(d["seed"]) != seed:
        return None
    n = int(d["histories"])
    if "sum" in d.files:
        return n, d["sum"].ravel(), d["sum2"].ravel()
    m, v = d["mean"].ravel(), d["var"].ravel()
    return n, n * m, n * (v * (n - 1) + m * m)


def make(name: str, threads: int, parts: int = 40, extend: bool = False) -> str:
    import oracle
    from paper_2510_24154_amd import synth
    g = GOLDENS[name]
    cfg = synth.narrow_field(field=g["field"], npx=g["npx"])
    P = oracle.Prepared(cfg, g["seed"])
    out = os.path.join(HERE, name + ".npz")
    n = g["histories"]
    start, s, s2 = 0, np.zeros(P.npix), np.zeros(P.npix)
    if extend:
        old = stored_sums(out, g["seed"])
        if old is not None and old[0] <= n:
            start, s, s2 = old
            s, s2 = s.copy(), s2.copy()
            print(f"[{name}] extending {start} stored histories to {n}", flush=True)
    m = max(1, (n - start) // parts)
    t0 = time.time()
    first = start
    while first < n:   # in parts, to report progress; the sums are the same
        cnt = min(m, n - first)
        _, _, si, s2i, _ = oracle.run(cfg, cnt, seed=g["seed"], first=first, threads=threads, prepared=P)
        s += si
        s2 += s2i
        first += cnt
        print(f"[{name}] {first}/{n} histories, {time.time() - t0:.0f} s", flush=True)
    mean = s / n
    var = np.maximum((s2 / n - mean * mean) / (n - 1), 0.0)
    np.savez_compressed(out, mean=mean.reshape(P.shape), var=var.reshape(P.shape), sum=s.reshape(P.shape),
                        sum2=s2.reshape(P.shape), histories=n, seed=g["seed"], field_cm=g["field"], npx=g["npx"],
                        pitch_cm=0.039, oracle_sha=oracle_source_sha())
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=list(GOLDENS), default=None)
    ap.add_argument("--extend", action="store_true")
    a = ap.parse_args()
    for name in ([a.only] if a.only else list(GOLDENS)):
        print(make(name, a.threads, extend=a.extend), flush=True)
