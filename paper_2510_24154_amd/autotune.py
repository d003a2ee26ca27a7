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
