"""Benchmark of the EPID transit Monte Carlo hot path on one MI355X.

Workload (one "step"): the coupled photon-electron configuration -- 1e8 histories
from a seeded 6 MV-like spectrum through a 256x256x128 phantom of 2 mm voxels (HU
from seeded water/lung/bone ellipsoids, 3 materials) into a 4-layer EPID with a
1024x768 image of 0.39 mm pixels, FP32 transport, FP64 tally, 64 variance batches.
Inputs are resident in HBM before timing; the timed region is K full runs.

Prints one JSON line: histories/s (whole job), the extrapolated time to 1% mean
relative uncertainty, the roofline figure of the dominant kernel (live HIP-event
durations from the engine's profiling mode), and the oracle timed on host cores
over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HISTORIES = 100_000_000
BATCHES = 64
CHUNK = 1 << 27   # one chunk per 1e8-history step: fewer queue passes and launch tails
# peak plain-ALU issue rate of MI355X: 256 CUs x 64 lanes x 2.4 GHz (one VALU op per lane per
# clock; FMA and packed FP32 doubling excluded because the hot path is not FMA-bound)
ALU_PEAK_OPS = 256 * 64 * 2.4e9
# algorithmic VALU lane-operations per unit of work ("Roofline")
OPS_PER_UNIT = {"electron_step": 310, "woodcock_step": 120, "epid_photon_step": 130}
KIND = ["photon_phantom", "electron_phantom", "photon_epid", "electron_epid"]
KERNEL = ["k_photon_phantom", "k_electron<phantom>", "k_photon_epid", "k_electron<epid>"]


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("csrc/kernels.hip", "csrc/device.hpp", "csrc/engine.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2510_24154_amd", f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload):
    """HBM bytes per unit of work of `kernel` from the committed rocprofv3 counter summaries
    (FETCH_SIZE and WRITE_SIZE passes, calibrated on a plain copy), or None when no summary
    was taken on the current kernel sources."""
    import glob
    sha = kernel_source_sha()
    key = f"traffic_bytes_per_unit[{kernel}]"
    wl = workload
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        for line in open(f):
            parts = line.strip().split(": ", 1)
            if len(parts) == 2:
                kv[parts[0]] = parts[1]
        if kv.get("source_sha") == sha and kv.get("workload") == wl and key in kv:
            return float(kv[key]), os.path.basename(f)
    return None, None


# workloads: the default benchmark line is "coupled"; the two segmented fields deliver the
# whole field (history ids [0, total)) in every step
WORKLOADS = {
    "coupled": ("coupled 6MV-like spectrum, 256x256x128 HU phantom (water/lung/bone), "
                "4-layer EPID 1024x768 @0.39 mm, 1e8 histories per step", HISTORIES),
    "imrt40": ("40-segment IMRT-like field (60 leaf pairs, uneven counts 1e6-5e7), same phantom and EPID "
               "as coupled, 3e8 histories per step", 300_000_000),
    "large60": ("60-segment field on a 512x512x200 anthropomorphic-like phantom of 1 mm voxels, "
                "4-layer EPID 1024x768, 2e9 histories per step", 2_000_000_000),
}


def smoothed_sigma_bar(eng, torch, k=15, thr=0.5):
    """sigma-bar for extrapolation from a noisy image: the pixel set (D >= thr * max D) and
    each pixel's D are taken from the k x k box mean of the image, each pixel's sigma from
    its own batch estimate.  Thresholding the raw image at a few tens of percent noise keeps
    the pixels that fluctuated upwards and understates sigma-bar."""
    m, v = eng.image()
    ms = torch.nn.functional.avg_pool2d(m[None, None], k, stride=1, padding=k // 2,
                                        count_include_pad=False)[0, 0]
    sel = ms >= thr * ms.max()
    return float((v[sel].clamp_min(0).sqrt() / ms[sel]).mean())


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="coupled")
    ap.add_argument("--histories", type=int, default=None,
                    help="histories per step (default: the workload's; a segmented field is rescaled)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3_000_000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--t1-measured", action="store_true",
                    help="also run the coupled workload until sigma-bar <= 1% (about 80 s) and time it")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; a run on N GPUs would shard histories "
                                   "by id and all-reduce the tallies (see DESIGN.md), which is not built"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2510_24154_amd as E
    from paper_2510_24154_amd import synth

    desc, n_default = WORKLOADS[a.workload]
    n_step = a.histories or n_default
    segmented = a.workload != "coupled"
    if a.workload == "coupled":
        cfg = synth.coupled_hetero()
    elif a.workload == "imrt40":
        cfg = synth.imrt_field()
    else:
        cfg = synth.large_anthropomorphic()
    if segmented and n_step != n_default:
        cfg = synth.with_histories_scaled(cfg, n_step)
    eng = E.Engine(0, seed=1).configure(cfg, batches=BATCHES, max_chunk=min(CHUNK, n_step))
    eng.bind()
    eng.set_profiling(True)
    h = 0
    for _ in range(a.warmup):
        eng.run(n_step, first=h)
        h = 0 if segmented else h + n_step
    eng.reset()
    torch.cuda.synchronize()
    first = h
    t0 = time.perf_counter()
    for i in range(a.steps):
        if segmented and i > 0:
            eng.reset()   # the same field again: sigma-bar and the counters describe one delivery
        eng.run(n_step, first=h)
        h = 0 if segmented else h + n_step
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = a.steps * n_step
    sb = eng.sigma_bar(0.5)
    c = eng.counters()
    value = n / dt
    # time to 1%: one delivery's sigma-bar scaled by 1/sqrt(N)
    t_n = dt / a.steps if segmented else dt
    t1 = t_n * (sb / 0.01) ** 2 if sb > 0 else None
    sb_s = smoothed_sigma_bar(eng, torch)
    t1_s = t_n * (sb_s / 0.01) ** 2 if sb_s > 0 else None

    # roofline of the dominant kernel: algorithmic lane-ops per launch / average launch time
    units = {1: c["e_steps_phantom"], 0: c["woodcock_steps"], 2: c["epid_photon_steps"], 3: c["e_steps_epid"]}
    per = {1: OPS_PER_UNIT["electron_step"], 0: OPS_PER_UNIT["woodcock_step"], 2: OPS_PER_UNIT["epid_photon_step"],
           3: OPS_PER_UNIT["electron_step"]}
    dom = max(range(4), key=lambda k: c["kernel_ms"][k])
    launches = max(1, c["kernel_launches"][dom])
    avg_s = c["kernel_ms"][dom] / 1e3 / launches
    ops_per_launch = units[dom] * per[dom] / launches
    achieved = ops_per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    kname = KERNEL[dom]
    per_unit, tsrc = profiled_traffic(kname, a.workload)
    traffic = per_unit * units[dom] / launches if per_unit else None
    roof = {"bound": "alu", "kernel": kname,
            "achieved": round(achieved, 3), "peak": round(ALU_PEAK_OPS / 1e12, 3), "unit": "Tlane-op/s",
            "frac": round(achieved * 1e12 / ALU_PEAK_OPS, 4),
            "traffic": round(traffic) if traffic else None, "traffic_unit": "bytes/launch",
            "traffic_source": tsrc,
            "traffic_GBps": round(traffic / avg_s / 1e9, 1) if traffic and avg_s > 0 else None,
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": launches,
            "unit_of_work": "electron condensed-history step" if dom in (1, 3) else KIND[dom],
            "units_per_launch": round(units[dom] / launches), "ops_per_unit": per[dom],
            "lane_utilisation": round(c["lane_iters"][dom] / max(1, c["wave_iters"][dom]), 4)}

    # the dose-response correction of the image (Sec. 2.2 and 3.1): radiological-thickness map,
    # field size and k(t, s) from Table 1, timed with HIP events on the engine's stream
    t_nodes, s_nodes, ktab = synth.response_table_1()
    s_eq = eng.field_size()
    img, _ = eng.image()
    th = eng.radiological_thickness()
    eng.dose_response(img, th, s_eq, t_nodes, s_nodes, ktab)
    torch.cuda.synchronize()
    reps = 20
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        th = eng.radiological_thickness()
    e1.record()
    for _ in range(reps):
        corrected = eng.dose_response(img, th, s_eq, t_nodes, s_nodes, ktab)
    e2.record()
    torch.cuda.synchronize()
    npix = img.numel()
    rt_ms, kr_ms = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
    response = {"field_size_cm": round(s_eq, 4), "rays": npix, "radiological_thickness_ms": round(rt_ms, 4),
                "rays_per_s": round(npix / (rt_ms * 1e-3), 1), "k_correction_ms": round(kr_ms, 4),
                "thickness_cm_range": [round(float(th.min()), 3), round(float(th.max()), 3)],
                "corrected_over_plain": round(float(corrected.sum() / img.sum()), 5)}

    measured = None
    if a.t1_measured and segmented:
        print("--t1-measured runs on the coupled workload only (a field's ids end at its total)", file=sys.stderr)
    elif a.t1_measured:
        # time to a 1% image measured directly: fresh tally, steps of 2e9 histories (ids
        # continue past 2^32), sigma-bar checked after each step
        eng.set_profiling(False)
        eng.reset()
        torch.cuda.synchronize()
        step = 2_000_000_000
        tm = time.perf_counter()
        done, sb1 = eng.run_until(0.01, thr=0.5, first=h, step=step, max_hist=1_000_000_000_000)
        torch.cuda.synchronize()
        tmd = time.perf_counter() - tm
        measured = {"s_to_1pct": round(tmd, 2), "histories": done, "sigma_bar": round(sb1, 5),
                    "sigma_bar_10pct": round(eng.sigma_bar(0.1), 5), "step_histories": step,
                    "first_history": h}
        print(json.dumps({"t1pct_measured": measured}), file=sys.stderr, flush=True)

    if a.calib_copy:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    cpu = None
    if not a.no_cpu_baseline and a.workload == "coupled":
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        ns = a.cpu_sample
        tc = time.perf_counter()
        oracle.run(cfg, ns, seed=1001, first=0, threads=threads)
        tcd = time.perf_counter() - tc
        # the same oracle on one core, over a tenth of the sample
        n1 = max(1000, ns // 10 // max(1, threads // 8))
        t1c = time.perf_counter()
        oracle.run(cfg, n1, seed=1001, first=0, threads=1)
        t1d = time.perf_counter() - t1c
        cpu = {"value": round(ns / tcd, 1), "unit": "histories/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} histories of the same workload (ids 0..{ns - 1}), {tcd:.1f} s wall on {threads} threads",
               "value_1core": round(n1 / t1d, 1),
               "sample_1core": f"{n1} histories (ids 0..{n1 - 1}), {t1d:.1f} s on 1 thread"}

    out = {
        "metric": "photon histories/s (coupled transport to a 1% EPID image)",
        "value": round(value, 1),
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": a.workload,
                   "histories_per_step": n_step, "batches": BATCHES, "tally": "fp64",
                   "first_history": first, "chunk": min(CHUNK, n_step)},
        "s_to_1pct_extrapolated": round(t1_s, 2) if t1_s else None,
        "s_to_1pct_extrapolated_raw_selection": round(t1, 2) if t1 else None,
        "sigma_bar_smoothed_selection": round(sb_s, 5),
        "sigma_bar_at_N": round(sb, 5),
        "N_for_sigma_bar": n_step if segmented else n,
        "roofline": roof,
        "cpu_baseline": cpu,
        "dose_response": response,
        "t1pct_measured": measured,
        "counters": {k: c[k] for k in ("woodcock_steps", "e_steps_phantom", "e_steps_epid", "epid_photon_steps",
                                       "tally_deposits", "launches", "kernel_ms", "kernel_launches",
                                       "queue_items", "lane_iters", "wave_iters")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
