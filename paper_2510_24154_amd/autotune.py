"""Autotuner of the engine's launch configuration: the number of histories processed
together (the chunk, which sets every queue's capacity and so the workspace size).  Larger
chunks mean fewer queue passes and launch tails per history but a larger workspace; the
best size depends on the workload and the free device memory.  Each candidate that fits is
bound and timed on the same histories; the fastest wins."""
from __future__ import annotations

import time

DEFAULT_CHUNKS = (1 << 23, 1 << 24, 1 << 25, 1 << 26, 1 << 27)


def tune_chunk(cfg, histories, candidates=DEFAULT_CHUNKS, seed=1, batches=64, mem_fraction=0.8, device=0,
               first=0):
    """Return (best chunk, {chunk: histories/s}) for a workload configuration.  A candidate is
    skipped when its workspace exceeds mem_fraction of the free device memory, or when it is
    more than twice the histories per run (it would only add workspace).  Every candidate
    runs the same history ids (one untimed warm-up run, then one timed run)."""
    import torch

    from . import Engine
    free, _ = torch.cuda.mem_get_info(device)
    rates = {}
    eng = Engine(device, seed)
    for chunk in sorted(candidates):
        if chunk > 2 * histories and rates:
            break
        eng.configure(cfg, batches=batches, max_chunk=int(min(chunk, histories)))
        if eng.workspace_size() > mem_fraction * free:
            break
        eng.bind()
        eng.run(histories, first=first)
        eng.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        eng.run(histories, first=first)
        torch.cuda.synchronize()
        rates[chunk] = histories / (time.perf_counter() - t)
        eng.ws = None   # release the workspace before the next candidate binds
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info(device)
    if not rates:
        raise RuntimeError("no chunk size fits in device memory")
    best = max(rates, key=rates.get)
    return best, rates


def _time_run(eng, histories, first, reps=1):
    import torch
    eng.reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        eng.run(histories, first=first)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tune(cfg, histories, candidates=DEFAULT_CHUNKS, seed=1, batches=64, mem_fraction=0.8, device=0, first=0,
         ipls=(1, 2, 4), pass_modes=(0, -1)):
    """Launch configuration for a workload: chunk size, items per lane and pass mode.

    Chunk: the run time of N histories is modelled as T(c) = a * ceil(N / c) + b (a the cost of
    one chunk: its source, fold and the launch tails of its queue passes; b the per-history
    work).  Three chunk sizes that fit in memory are timed (the smallest, the middle and the
    largest), (a, b) is fitted by least squares, and the candidate with the smallest predicted
    time wins (the smaller workspace on a tie).  Then, at that chunk, every pair of items per
    lane (grid sizing) and pass mode (0: host-driven passes, -1: device-driven) is timed and the
    fastest kept.  Returns a dict with the choice, the timings and the fitted model."""
    import numpy as np
    import torch

    from . import Engine
    free, _ = torch.cuda.mem_get_info(device)
    eng = Engine(device, seed)
    fits = []
    for chunk in sorted(candidates):
        c = int(min(chunk, histories))
        if fits and c == fits[-1]:
            break
        eng.configure(cfg, batches=batches, max_chunk=c)
        if eng.workspace_size() > mem_fraction * free:
            break
        fits.append(c)
    if not fits:
        raise RuntimeError("no chunk size fits in device memory")
    probe = sorted({fits[0], fits[len(fits) // 2], fits[-1]})
    measured = {}
    for c in probe:
        eng.configure(cfg, batches=batches, max_chunk=c)
        eng.bind()
        eng.set_passes(0, 2)
        eng.run(histories, first=first)                 # warm-up
        measured[c] = _time_run(eng, histories, first)
        eng.ws = None
        torch.cuda.empty_cache()
    x = np.array([float(-(-histories // c)) for c in probe])
    y = np.array([measured[c] for c in probe])
    if len(probe) >= 2 and np.ptp(x) > 0:
        a, b = np.polyfit(x, y, 1)
    else:
        a, b = 0.0, float(y.mean())
    predicted = {c: float(a * -(-histories // c) + b) for c in fits}
    best_chunk = min(fits, key=lambda c: (round(predicted[c], 6), c))
    eng.configure(cfg, batches=batches, max_chunk=best_chunk)
    eng.bind()
    launch = {}
    for ipl in ipls:
        for pm in pass_modes:
            eng.set_passes(pm, ipl)
            eng.run(histories, first=first)             # warm-up (a device-driven run learns its passes)
            launch[(ipl, pm)] = _time_run(eng, histories, first)
    (best_ipl, best_pm) = min(launch, key=launch.get)
    eng.ws = None
    torch.cuda.empty_cache()
    return {"chunk": best_chunk, "items_per_lane": best_ipl, "device_passes": best_pm,
            "model": {"s_per_chunk": float(a), "s_fixed": float(b)},
            "chunk_s_measured": {int(k): round(v, 6) for k, v in measured.items()},
            "chunk_s_predicted": {int(k): round(v, 6) for k, v in predicted.items()},
            "launch_s": {f"ipl{k[0]}_passes{k[1]}": round(v, 6) for k, v in launch.items()}}
