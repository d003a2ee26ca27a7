"""Benchmark of the EPID transit Monte Carlo hot path on one MI355X.

Workload (one "step"): one delivery of a 40-segment IMRT-like field -- seeded MLC
apertures of 60 leaf pairs with uneven history counts (1e6-5e7, 3e8 in all) from a
seeded 6 MV-like spectrum through a 256x256x128 phantom of 2 mm voxels (HU from seeded
water/lung/bone ellipsoids, 3 materials) into a 4-layer EPID with a 1024x768 image of
0.39 mm pixels, FP32 transport, FP64 tally, 64 variance batches.  `--workload coupled`
runs the single 10x10 cm open field at 1e8 histories per step instead.  Inputs are
resident in HBM before timing; the timed region is K full runs.

Prints one JSON line: histories/s (whole job), the time to 1% mean relative uncertainty
extrapolated by 1/sqrt(N) from one delivery, the roofline figures of the dominant kernel
(live HIP-event durations from the engine's profiling mode) against the ALU issue rate and
against the gather, bandwidth and atomic peaks measured on the same GPU by the library's
probes, and the oracle timed on the host's cores over a bounded sample of the workload.
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
# algorithmic VALU lane-operations per unit of work, counted from the step formulas
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


# workloads: the default benchmark line is "imrt40"; the segmented fields deliver the whole
# field (history ids [0, total)) in every step
WORKLOADS = {
    "coupled": ("coupled 6MV-like spectrum, 256x256x128 HU phantom (water/lung/bone), "
                "4-layer EPID 1024x768 @0.39 mm, 1e8 histories per step", HISTORIES),
    "imrt40": ("40-segment IMRT-like field (60 leaf pairs, uneven counts 1e6-5e7), same phantom and EPID "
               "as coupled, 3e8 histories per step", 300_000_000),
    "large60": ("60-segment field on a 512x512x200 anthropomorphic-like phantom of 1 mm voxels, "
                "4-layer EPID 1024x768, 2e9 histories per step", 2_000_000_000),
    "imrt40_2p5mm": ("the 40-segment IMRT-like field scaled to 1e9 histories onto a 160x160 image of 2.5 mm "
                     "pixels (the pixel pitch and history count the paper quotes its timing at)", 1_000_000_000),
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


DN_LOW, DN_HIGH, DN_REF = 2_000_000, 200_000_000, 10_000_000_000
DN_PLAIN = (2_000_000, 20_000_000, 200_000_000, 2_000_000_000)
DN_FLOP = 0.2136e12   # forward FLOPs of the network per 1024 x 768 image (2 x multiply-adds)
BF16_PEAK = 2.5e15    # dense BF16 MFMA, MI355X


def dn_hbm_bytes(px=1024 * 768):
    """Compulsory HBM bytes of one forward pass over `px` pixels: each layer's input read and
    output written once (BF16 NHWC, c_l = 32 * 2^l channels at 1/4^l of the pixels), the
    pooled and upsampled tensors, the 8-channel input (16 B per pixel) built from the two FP64
    planes, the frame sum, and the head, which runs in the last convolution's epilogue: that
    convolution's 32-channel output never reaches HBM, the head reads the FP32 image channel
    and writes the FP64 output."""
    P = lambda l: px // 4 ** l
    c = lambda l: 32 * 2 ** l
    b = px * 8 + px * (8 + 8 + 16 + 4)
    for l in range(4):
        b += (px * 16 if l == 0 else P(l) * c(l - 1) * 2) + P(l) * c(l) * 2
        b += 2 * P(l) * c(l) * 2 + (P(l + 1) * c(l) * 2 if l < 3 else 0)
    for l in (2, 1, 0):
        b += P(l + 1) * c(l + 1) * 2 + P(l) * c(l) * 2
        b += P(l) * 2 * c(l) * 2 + P(l) * c(l) * 2 + (2 if l > 0 else 1) * P(l) * c(l) * 2
    return b + px * (4 + 8)


DN_HBM_BYTES = dn_hbm_bytes()   # 9.06e8 for 1024 x 768


def error_regions(ref, evl, gmap, sel):
    """Where an image's error sits, against the reference on the same binned grid: the ratio of
    the in-field sums (a global scale error), and the mean signed relative error, the relative
    RMSE and the fraction of gamma failures on flat pixels and on pixels of steep gradient,
    where a 2 mm shift moves the reference by more than 2% of its maximum (penumbrae and
    leaf edges)."""
    import numpy as np
    gy, gx = np.gradient(ref)
    steep = np.hypot(gx, gy) * (0.2 / 0.312) > 0.02 * ref.max()
    out = {"sum_ratio": round(float(evl[sel].sum() / ref[sel].sum()), 4)}
    for name, m in (("flat", sel & ~steep), ("steep", sel & steep)):
        if not m.any():
            continue
        rel = (evl[m] - ref[m]) / ref[m]
        out[name] = {"pixels": int(m.sum()), "mean_rel_err": round(float(rel.mean()), 4),
                     "rel_rmse": round(float(np.sqrt(np.mean(rel ** 2))), 4),
                     "gamma_fail": round(float(np.mean(gmap[m] > 1.0)), 4)}
    return out


def denoiser_section(a, E, torch):
    """Train the denoiser on engine-generated full-size fields (by default the stated recipe:
    500 fields, 2e6 histories in, 2e8 as target), then on held-out fields compare the denoised
    low-count image and plain images of 2e6..2e9 histories with a 1e10-history image on 8 x
    8-binned pixels (3.1 mm): 2%/2 mm gamma (global, 10% threshold), the in-field relative
    RMSE and where the denoised error sits, timing each path end to end (transport, image,
    thickness map and network pass).  With --dn-seeds K, K networks are trained from
    different initial weights and crop orders on the same pairs and judged on the same
    images."""
    import numpy as np

    from paper_2510_24154_amd import denoise as D
    from paper_2510_24154_amd import synth
    from tests._stats import gamma_map, rebin
    out = {}
    sync = torch.cuda.synchronize
    t = time.perf_counter()
    fields = [synth.denoise_field(s, mixed=bool(a.dn_mixed)) for s in range(a.dn_fields)]
    out["train_recipe"] = "mixed: single-segment ellipsoid fields and multi-segment thorax fields" if a.dn_mixed \
        else "single-segment ellipsoid fields"
    n_low = int(a.dn_low)
    low, high, th = D.make_pairs(fields, n_low, int(a.dn_target), seed=17, max_chunk=1 << 26, report=50)
    out["input_histories"] = n_low
    out["train_target_histories"] = int(a.dn_target)
    out["train_fields"] = a.dn_fields
    out["train_data_s"] = round(time.perf_counter() - t, 2)
    print(f"[denoiser] {a.dn_fields} training pairs in {out['train_data_s']} s", file=sys.stderr, flush=True)

    # held-out fields: the noisy input and its thickness map, plain images, the reference
    eng = E.Engine(0, seed=29)
    evals = []
    for i in range(a.dn_eval):
        cfg = synth.denoise_field(100_000 + i)
        eng.configure(cfg, batches=64, max_chunk=1 << 26)
        eng.bind()
        f = {"cfg": cfg, "plain": {}, "plain_s": {}}
        eng.reset()
        eng.run(n_low, first=0)
        f["img"] = eng.image()[0][None].clone()
        f["tk"] = eng.radiological_thickness()[None].clone()
        first = n_low
        for n in DN_PLAIN:
            eng.reset()
            sync()
            t = time.perf_counter()
            eng.run(n, first=first)
            m = eng.image()[0]
            sync()
            f["plain_s"][f"plain_{n:.0e}"] = time.perf_counter() - t
            f["plain"][f"plain_{n:.0e}"] = m.cpu().numpy()
            first += n
        eng.reset()
        eng.run(DN_REF, first=first)
        f["ref"] = rebin(eng.image()[0].cpu().numpy(), 8)
        f["sel"] = f["ref"] >= 0.1 * f["ref"].max()
        evals.append(f)

    def judge(img):
        """gamma, RMSE, error regions of a full-size image against each held-out reference"""
        res = []
        for f, im in zip(evals, img):
            b = rebin(im, 8)
            g = gamma_map(f["ref"], b, 0.312, dd=0.02, dta=0.2)
            sel = f["sel"]
            res.append({"gamma": float(np.mean(g[sel] <= 1.0)),
                        "rmse": float(np.sqrt(np.mean((b[sel] - f["ref"][sel]) ** 2)) / f["ref"][sel].mean()),
                        "regions": error_regions(f["ref"], b, g, sel)})
        return res

    plain_res = {k: judge([f["plain"][k] for f in evals]) for k in evals[0]["plain"]}
    seeds = []
    full = None
    for sd in range(a.dn_seeds):
        net = D.Unet(0).bind(8, 256, 256)
        net.set_params(synth.unet_params(net.shapes(), seed=1 + sd, head_scale=0.01))
        net.set_ema(a.dn_ema)
        sync()
        t = time.perf_counter()
        losses = D.train(net, low, high, th, steps=a.dn_steps, batch=8, crop=256, lr=2e-3, lr_end=1e-4, seed=3 + sd,
                         report=max(1, a.dn_steps // 4))
        sync()
        dt = time.perf_counter() - t
        fn = D.Unet(0).bind(1, 1024, 768)
        fn.set_params(net.get_ema_params() if a.dn_ema > 0 else net.get_params())
        del net
        dens, dens_r, times = [], [], []
        for f in evals:
            # the denoised path end to end: 2e6 histories, the thickness map, one network pass
            eng.configure(f["cfg"], batches=64, max_chunk=1 << 26)
            eng.bind()
            for rep in range(2):   # the first pass warms the kernels up
                eng.reset()
                sync()
                t1 = time.perf_counter()
                eng.run(n_low, first=0)
                img = eng.image()[0][None]
                tk = eng.radiological_thickness()[None]
                den = fn.forward(img, tk)
                sync()
                dts = time.perf_counter() - t1
            times.append(dts)
            dens.append(den[0].cpu().numpy())
            # the same image rescaled to the noisy input's sum, an unbiased estimate of the
            # field's integral (flux-preserving): separates a global scale error from local ones
            dens_r.append(dens[-1] * float(img.sum() / den.sum()))
        r = judge(dens)
        rr = judge(dens_r)
        row = {"seed": sd, "train_s": round(dt, 2), "loss_first_last": [round(float(losses[:50].mean()), 4),
                                                                           round(float(losses[-50:].mean()), 4)],
               "gamma": round(float(np.mean([x["gamma"] for x in r])), 4),
               "rmse": round(float(np.mean([x["rmse"] for x in r])), 4),
               "denoised_s": round(float(np.mean(times)), 4),
               "gamma_rescaled": round(float(np.mean([x["gamma"] for x in rr])), 4),
               "rmse_rescaled": round(float(np.mean([x["rmse"] for x in rr])), 4),
               "regions": [x["regions"] for x in r]}
        seeds.append(row)
        print(f"[denoiser] seed {sd}: gamma {row['gamma']} rmse {row['rmse']} in {row['denoised_s']} s", file=sys.stderr,
              flush=True)
        if full is None:
            full = fn
            out["train_steps"] = a.dn_steps
            out["train_s"] = round(dt, 2)
            out["train_TFLOPs"] = round(3 * DN_FLOP * 8 * 65536 / 786432 * a.dn_steps / dt / 1e12, 1)
            out["loss_first_last"] = row["loss_first_last"]
            out["weight_ema_decay"] = a.dn_ema
            out["eval_regions_denoised"] = row["regions"]
    del low, high, th
    out["eval_fields"] = a.dn_eval
    out["gamma_2pct_2mm"] = {"denoised": seeds[0]["gamma"], "denoised_rescaled": seeds[0]["gamma_rescaled"]}
    out["in_field_rel_rmse"] = {"denoised": seeds[0]["rmse"], "denoised_rescaled": seeds[0]["rmse_rescaled"]}
    for k, r in plain_res.items():
        out["gamma_2pct_2mm"][k] = round(float(np.mean([x["gamma"] for x in r])), 4)
        out["in_field_rel_rmse"][k] = round(float(np.mean([x["rmse"] for x in r])), 4)
    out["eval_regions_plain"] = {k: r[0]["regions"] for k, r in plain_res.items()}
    if a.dn_seeds > 1:
        g = np.array([x["gamma"] for x in seeds])
        e = np.array([x["rmse"] for x in seeds])
        out["seeds"] = {"n": a.dn_seeds, "gamma_mean": round(float(g.mean()), 4), "gamma_sd": round(float(g.std(ddof=1)), 4),
                        "rmse_mean": round(float(e.mean()), 4), "rmse_sd": round(float(e.std(ddof=1)), 4),
                        "per_seed": [{k: v for k, v in x.items() if k != "regions"} for x in seeds]}
    secs = {k: float(np.mean([f["plain_s"][k] for f in evals])) for k in evals[0]["plain_s"]}
    secs["denoised"] = seeds[0]["denoised_s"]
    out["seconds"] = {k: round(v, 4) for k, v in secs.items()}
    rm = dict(out["in_field_rel_rmse"])
    n_eq, sp, e_ref2 = equal_rmse(rm, secs, rm["denoised"], secs["denoised"])
    if n_eq:
        out["plain_histories_at_equal_rmse"] = float(f"{n_eq:.3g}")
        out["speedup_at_equal_rmse"] = round(sp, 1)
    out["reference_rmse_share"] = round(float(np.sqrt(e_ref2)), 4)
    # plain histories needed for the denoised pass rate: the smallest plain N that reaches it
    g_den = out["gamma_2pct_2mm"]["denoised"]
    match = [n for n in DN_PLAIN if out["gamma_2pct_2mm"][f"plain_{n:.0e}"] >= g_den]
    if match:
        n = match[0]
        out["plain_histories_at_equal_gamma"] = n
        out["speedup_at_equal_gamma"] = round(secs[f"plain_{n:.0e}"] / secs["denoised"], 1)
    else:
        out["plain_histories_at_equal_gamma"] = f"> {DN_PLAIN[-1]:.0e}"
        out["speedup_at_equal_gamma"] = f"> {secs[f'plain_{DN_PLAIN[-1]:.0e}'] / secs['denoised']:.1f}"

    # the large case: anthropomorphic-like phantom of 1 mm voxels and a 60-segment field, both
    # unlike the training fields; every image is a whole delivery of the field scaled to its
    # history count, and the reference comes from an engine with another seed
    if a.dn_large:
        base = synth.large_anthropomorphic(total=DN_REF)
        big = {}
        for label, n, seed in [("ref", DN_REF, 31), ("low", n_low, 29)] + [(f"plain_{m:.0e}", m, 29) for m in DN_PLAIN]:
            e2 = E.Engine(0, seed=seed)
            e2.configure(synth.with_histories_scaled(base, n), batches=64, max_chunk=1 << 26)
            e2.bind()
            sync()
            t = time.perf_counter()
            e2.run(n, first=0)
            img_l = e2.image()[0]
            if label == "low":
                tk = e2.radiological_thickness()[None]
                d = full.forward(img_l[None], tk)
                sync()
                big["denoised_s"] = time.perf_counter() - t
                big["denoised"] = d[0].cpu().numpy()
            else:
                sync()
                big[label + "_s"] = time.perf_counter() - t
                big[label] = img_l.cpu().numpy()
            del e2
        ref = rebin(big.pop("ref"), 8)
        big.pop("ref_s")
        sel = ref >= 0.1 * ref.max()
        lg = {"gamma_2pct_2mm": {}, "in_field_rel_rmse": {}, "seconds": {}}
        for k, v in big.items():
            if k.endswith("_s"):
                lg["seconds"][k[:-2]] = round(v, 4)
                continue
            b = rebin(v, 8)
            gm = gamma_map(ref, b, 0.312, dd=0.02, dta=0.2)
            lg["gamma_2pct_2mm"][k] = round(float(np.mean(gm[sel] <= 1.0)), 4)
            lg["in_field_rel_rmse"][k] = round(float(np.sqrt(np.mean((b[sel] - ref[sel]) ** 2)) / ref[sel].mean()), 4)
            if k == "denoised":
                lg["regions_denoised"] = error_regions(ref, b, gm, sel)
        n_eq, sp, _ = equal_rmse(lg["in_field_rel_rmse"], lg["seconds"], lg["in_field_rel_rmse"]["denoised"],
                                 lg["seconds"]["denoised"])
        if n_eq:
            lg["plain_histories_at_equal_rmse"] = float(f"{n_eq:.3g}")
            lg["speedup_at_equal_rmse"] = round(sp, 1)
        out["large_case"] = lg
        print(f"[denoiser] large case: {lg}", file=sys.stderr, flush=True)
    # inference throughput of the network alone
    x = evals[0]["img"].clone()
    for _ in range(3):
        full.forward(x, x)
    sync()
    t = time.perf_counter()
    for _ in range(20):
        full.forward(x, x)
    sync()
    f_ms = (time.perf_counter() - t) / 20 * 1e3
    out["inference_ms"] = round(f_ms, 3)
    # the same pass replayed from a HIP graph (one launch for the whole network)
    y = torch.empty_like(x)
    graph = full.capture_forward(x, x, y)
    for _ in range(3):
        graph.replay()
    sync()
    t = time.perf_counter()
    for _ in range(20):
        graph.replay()
    sync()
    out["inference_graph_ms"] = round((time.perf_counter() - t) / 20 * 1e3, 3)
    # the pass does 0.2136 TFLOP on about 1.0 GB of compulsory HBM traffic (every layer's input
    # and output once, BF16 NHWC), 212 FLOP/B, under the machine balance of 2.5 PFLOP/s over
    # 8 TB/s (312 FLOP/B): its roofline is the memory one, and the MFMA fraction is also given
    gbps = DN_HBM_BYTES / (f_ms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(gbps, 1), "peak": 8000.0, "unit": "GB/s",
                       "frac": round(gbps / 8000.0, 4), "algorithmic_bytes": DN_HBM_BYTES,
                       "mfma_TFLOPs": round(DN_FLOP / (f_ms * 1e-3) / 1e12, 1),
                       "mfma_frac": round(DN_FLOP / (f_ms * 1e-3) / BF16_PEAK, 4),
                       "scope": "whole forward pass, 1024 x 768, BF16 MFMA"}
    return out


def equal_rmse(rmse, seconds, denoised_rmse, denoised_s):
    """Plain histories with the denoised image's RMSE, and the wall-clock speedup: RMSE^2 =
    c / N + e_ref^2 fitted through the two largest plain counts (e_ref^2 is the reference's
    own share, common to every comparison), the plain rate from the largest run."""
    n_hi, n_lo = DN_PLAIN[-1], DN_PLAIN[-2]
    e2_hi, e2_lo = rmse[f"plain_{n_hi:.0e}"] ** 2, rmse[f"plain_{n_lo:.0e}"] ** 2
    c = (e2_lo - e2_hi) / (1.0 / n_lo - 1.0 / n_hi)
    e_ref2 = max(0.0, e2_hi - c / n_hi)
    d2 = denoised_rmse ** 2 - e_ref2
    if c <= 0 or d2 <= 0:
        return None, None, e_ref2
    n_eq = c / d2
    rate = n_hi / seconds[f"plain_{n_hi:.0e}"]
    return n_eq, n_eq / rate / denoised_s, e_ref2


def run_to_1pct(eng, torch, step, max_steps=20000):
    """Run from history id 0 until sigma-bar (pixels >= 50% of max) <= 1%, one check per
    `step` histories (the library's run-until loop, driven from here so that progress is
    printed every ~10 s); the wall time, histories and sigma-bars (the 10% selection too)."""
    torch.cuda.synchronize()
    tm = time.perf_counter()
    done, sb1, shown = 0, float("inf"), tm
    for _ in range(max_steps):
        eng.run(step, first=done)
        done += step
        sb1 = eng.sigma_bar(0.5)
        if sb1 <= 0.01:
            break
        if time.perf_counter() - shown > 10.0:
            shown = time.perf_counter()
            print(f"[t1] {done:.3e} histories, sigma-bar {sb1:.4f}, {shown - tm:.0f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tmd = time.perf_counter() - tm
    return {"s_to_1pct": round(tmd, 2), "histories": done, "sigma_bar": round(sb1, 5),
            "sigma_bar_10pct": round(eng.sigma_bar(0.1), 5), "step_histories": step,
            "histories_per_s": round(done / tmd, 1)}


def host_cpu():
    """The host's CPU facts: nproc, the CPUs this process may run on, the cgroup CPU quota
    (if any) and the lscpu model name."""
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        q = open("/sys/fs/cgroup/cpu.max").read().split()
        if q and q[0] != "max":
            info["cgroup_cpus"] = round(int(q[0]) / int(q[1]), 2)
    except (OSError, ValueError, IndexError):
        pass
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                info["model"] = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


# a GPU machine gives one GPU's worth of host CPUs to a run (16), whatever nproc reports
HOST_CPUS_PER_GPU = 16


def cpu_baseline(cfg, ns, field_total=None):
    """The oracle as it stands, timed on the host's cores over a bounded sample of the same
    workload: every CPU the run may use (at most one GPU's share of the host, 16), then one
    core over a tenth of the sample.  For a segmented field the sample is spread over the
    field: eight slices of ids starting at k/8 of its total, so every part of the delivery
    contributes."""
    import oracle
    host = host_cpu()
    threads = max(1, min(HOST_CPUS_PER_GPU, host["affinity"], int(host.get("cgroup_cpus", 1e9)) or 1))
    P = oracle.Prepared(cfg, 1001)
    slices = 8 if field_total else 1

    def timed(n, th):
        per = n // slices
        t = time.perf_counter()
        for k in range(slices):
            first = (k * field_total) // slices if field_total else 0
            oracle.run(cfg, per, seed=1001, first=first, threads=th, prepared=P)
        return per * slices, time.perf_counter() - t

    n_all, t_all = timed(ns, threads)
    n_one, t_one = timed(max(1000 * slices, ns // 10 // max(1, threads // 8)), 1)
    where = f"{slices} slices of ids spread over the field" if field_total else f"ids 0..{n_all - 1}"
    return {"value": round(n_all / t_all, 1), "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_all} histories of the same workload ({where}), {t_all:.1f} s wall on {threads} threads",
            "value_1core": round(n_one / t_one, 1),
            "sample_1core": f"{n_one} histories, {t_one:.1f} s on 1 thread",
            "host": host}


def peaks(E, torch, table_bytes):
    """The memory and atomic peaks of this GPU from the library's probes (epidmc_microbench),
    each timed with HIP events on torch's stream over 10 launches after one warm-up: a
    streaming copy of 2 GiB, random 4-byte gathers from a table of the phantom's size (and
    from 4 MiB and 1 GiB tables), FP64 and int64 atomic adds spread over 8 MiB or aimed at 64
    hot words."""
    buf = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    out = {}
    t = timed(lambda: E.microbench(E.MB_COPY, buf))
    out["copy_GBps"] = round(buf.numel() / t / 1e9, 1)   # half read, half written
    threads, per = 256 * 2048, 256
    bits = max(10, min(31, int(round(__import__("math").log2(max(1, table_bytes) / 4)))))
    for label, b in (("phantom", bits), ("4MiB", 20), ("1GiB", 28)):
        t = timed(lambda: E.microbench(E.MB_GATHER, buf, b, per, threads))
        out[f"gather_{label}_Gps"] = round(threads * per / t / 1e9, 2)
    out["gather_phantom_table_bytes"] = 4 << bits
    for kind, name in ((E.MB_ATOMIC_F64, "f64"), (E.MB_ATOMIC_I64, "i64")):
        t = timed(lambda: E.microbench(kind, buf, 20, 64, threads))
        out[f"atomic_{name}_spread_Gps"] = round(threads * 64 / t / 1e9, 3)
        t = timed(lambda: E.microbench(kind, buf, 6, 4, threads), reps=3)
        out[f"atomic_{name}_hot64_Gps"] = round(threads * 4 / t / 1e9, 3)
    del buf
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="imrt40")
    ap.add_argument("--histories", type=int, default=None,
                    help="histories per step (default: the workload's; a segmented field is rescaled)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=3_000_000)
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the segmented field replayed from one captured HIP graph (default on)")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="pick chunk size, items per lane and pass mode by timing the candidates that fit "
                         "(default on; --no-autotune: 2^27, 2, host-driven)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--no-denoiser", action="store_true",
                    help="skip training the denoiser on engine-generated fields and comparing it with plain MC")
    ap.add_argument("--dn-fields", type=int, default=500)
    ap.add_argument("--dn-steps", type=int, default=3000)
    ap.add_argument("--dn-target", type=float, default=DN_HIGH)
    ap.add_argument("--dn-low", type=float, default=DN_LOW)
    ap.add_argument("--dn-eval", type=int, default=3)
    ap.add_argument("--dn-seeds", type=int, default=1, help="networks trained from different seeds on the same pairs")
    ap.add_argument("--dn-large", type=int, default=1, help="also judge the denoiser on the large case (0: skip)")
    ap.add_argument("--dn-ema", type=float, default=0.0,
                    help="decay of the moving average of the weights used for inference (0: the last weights)")
    ap.add_argument("--dn-mixed", type=int, default=1,
                    help="1: every other training field is a thorax-like phantom under a multi-segment field")
    ap.add_argument("--t1-measured", action="store_true",
                    help="also run the workload until sigma-bar <= 1%% and time it (a segmented field is "
                         "delivered again with new history ids until then; about 150 s for imrt40)")
    ap.add_argument("--no-t1-accumulated", action="store_true",
                    help="skip the time to 1%% from an accumulated image (about 8 s of further deliveries after "
                         "the timed ones; for profiling runs whose counters should cover the timed work only)")
    ap.add_argument("--no-t1-paper", action="store_true",
                    help="skip the measured time to 1%% at the paper's pixel pitch (imrt40_2p5mm, about 35 s)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; a run on N GPUs would shard histories "
                                   "by id and all-reduce the tallies, which is not built"}))
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
    elif a.workload == "imrt40_2p5mm":
        cfg = synth.with_histories_scaled(synth.imrt_field(npx=(160, 160), pitch=0.25), n_default)
    else:
        cfg = synth.large_anthropomorphic()
    if segmented and n_step != n_default:
        cfg = synth.with_histories_scaled(cfg, n_step)
    chunk, tuned, ipl, dpasses = CHUNK, None, 2, 0
    if a.autotune:
        from paper_2510_24154_amd.autotune import tune
        tuned = tune(cfg, n_step, seed=1, batches=BATCHES)
        chunk, ipl, dpasses = tuned["chunk"], tuned["items_per_lane"], tuned["device_passes"]
        print(f"[autotune] {tuned}", file=sys.stderr, flush=True)
    eng = E.Engine(0, seed=1).configure(cfg, batches=BATCHES, max_chunk=min(chunk, n_step))
    eng.bind()
    eng.set_passes(dpasses, ipl)
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

    # the whole delivery replayed as one HIP graph (all segments, chunks, queue passes and folds
    # in one launch; no profiling events inside), timed separately from the measurement above
    graph = None
    if a.graph and segmented:
        eng.set_profiling(False)
        eng.reset()
        eng.run(n_step, first=0)            # an eager delivery: the pass counts the capture uses
        eng.set_graph(True)
        eng.reset()
        eng.run(n_step, first=0)            # capture and first replay
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(a.steps):
            eng.reset()
            eng.run(n_step, first=0)
        torch.cuda.synchronize()
        g_step = (time.perf_counter() - tg) / a.steps
        eng.set_graph(False)
        eng.set_profiling(True)
        graph = {"ms_per_step": round(g_step * 1e3, 3), "histories_per_s": round(n_step / g_step, 1),
                 "note": "whole field replayed from one captured graph; a reset per step as in the eager loop"}
        print(f"[graph] {graph}", file=sys.stderr, flush=True)

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

    # on-box peaks, then the dominant kernel's rates as fractions of them: voxel gathers per
    # second against random 4-byte gathers from a table of the phantom's size, its calibrated
    # memory traffic past L2 against the streaming copy (part of that traffic is served by the
    # Infinity Cache, which holds the phantom, so it can exceed the copy's HBM rate), and the
    # image tally's atomic adds per second of the step against spread FP64 atomics
    pk = peaks(E, torch, int(np.prod(cfg["phantom"]["shape"])) * 4)
    t_step = dt / a.steps
    gathers_ps = units[dom] / launches / avg_s if dom in (0, 1) and avg_s > 0 else None
    fractions = {
        "alu": roof["frac"],
        "gather": round(gathers_ps / (pk["gather_phantom_Gps"] * 1e9), 4) if gathers_ps else None,
        "past_l2_vs_copy": round(roof["traffic_GBps"] / pk["copy_GBps"], 4) if roof["traffic_GBps"] else None,
        "atomic": round(c["tally_deposits"] / (t_step if segmented else dt) / (pk["atomic_f64_spread_Gps"] * 1e9), 6),
    }
    fractions["binding"] = max((k for k in ("alu", "gather", "past_l2_vs_copy", "atomic") if fractions[k] is not None),
                               key=lambda k: fractions[k])
    roof["gathers_per_s"] = round(gathers_ps, 1) if gathers_ps else None

    # time to 1% from an accumulated image: one delivery's sigma-bar underestimates it, since
    # selecting the pixels >= 50% of a noisy image's maximum keeps pixels that fluctuated
    # upwards; K deliveries (about 8 s, new history ids each) bring the noise down to where
    # the selection has settled, and sigma-bar then falls as 1/sqrt(N)
    k_acc, t_acc, sb_acc, t1_acc = 0, None, None, None
    if not a.no_t1_accumulated:
        eng.set_profiling(False)
        eng.reset()
        torch.cuda.synchronize()
        k_acc = max(1, min(1000, int(round(8.0 / t_n))))
        ta = time.perf_counter()
        for k in range(k_acc):
            eng.run(n_step, first=k * n_step)
        torch.cuda.synchronize()
        t_acc = time.perf_counter() - ta
        sb_acc = eng.sigma_bar(0.5)
        t1_acc = t_acc * (sb_acc / 0.01) ** 2 if sb_acc > 0 else None

    measured = None
    if a.t1_measured:
        # time to a 1% image measured directly: fresh tally, sigma-bar checked after each step
        # (a segmented field: one whole delivery per step, history ids continuing past the
        # field's total, i.e. new independent deliveries; otherwise steps of 2e9 histories)
        eng.set_profiling(False)
        eng.reset()
        torch.cuda.synchronize()
        measured = run_to_1pct(eng, torch, n_step if segmented else 2_000_000_000)
        print(json.dumps({"t1pct_measured": measured}), file=sys.stderr, flush=True)
    del eng
    torch.cuda.empty_cache()
    paper_t1 = None
    if a.workload == "imrt40" and not a.no_t1_paper:
        cfg_p = synth.with_histories_scaled(synth.imrt_field(npx=(160, 160), pitch=0.25), 1_000_000_000)
        eng_p = E.Engine(0, seed=2).configure(cfg_p, batches=BATCHES, max_chunk=CHUNK)
        eng_p.bind()
        eng_p.set_passes(dpasses, ipl)
        paper_t1 = run_to_1pct(eng_p, torch, 1_000_000_000)
        paper_t1["workload"] = WORKLOADS["imrt40_2p5mm"][0]
        print(json.dumps({"t1pct_measured_at_paper_pitch": paper_t1}), file=sys.stderr, flush=True)
        del eng_p
        torch.cuda.empty_cache()

    dn = None
    if not a.no_denoiser:
        try:
            dn = denoiser_section(a, E, torch)
        except Exception as e:   # the transport line above must still be reported
            dn = {"error": f"{type(e).__name__}: {e}"}

    if a.calib_copy:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    cpu = None
    if not a.no_cpu_baseline and a.workload in ("coupled", "imrt40"):
        cpu = cpu_baseline(cfg, a.cpu_sample, n_default if segmented else None)
        print(f"[cpu_baseline] {cpu}", file=sys.stderr, flush=True)

    out = {
        "metric": "photon histories/s and s-to-1%-uncertainty EPID image; denoised vs plain at \u226599% gamma",
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
                   "first_history": first, "chunk": min(chunk, n_step), "items_per_lane": ipl,
                   "device_passes": dpasses, "autotune": tuned},
        "s_to_1pct_extrapolated": round(t1_acc, 2) if t1_acc else None,
        "sigma_bar_at_N": round(sb_acc, 5) if sb_acc is not None else None,
        "N_for_sigma_bar": k_acc * n_step if k_acc else None,
        "s_for_N": round(t_acc, 3) if t_acc is not None else None,
        "s_to_1pct_one_delivery": round(t1, 2) if t1 else None,
        "s_to_1pct_one_delivery_smoothed_selection": round(t1_s, 2) if t1_s else None,
        "sigma_bar_one_delivery": round(sb, 5),
        "sigma_bar_one_delivery_smoothed_selection": round(sb_s, 5),
        "roofline": roof,
        "graph_replay": graph,
        "roofline_fractions": fractions,
        "peaks": pk,
        "cpu_baseline": cpu,
        "dose_response": response,
        "t1pct_measured": measured,
        "t1pct_measured_at_paper_pitch": paper_t1,
        "denoiser": dn,
        "counters": {k: c[k] for k in ("woodcock_steps", "e_steps_phantom", "e_steps_epid", "epid_photon_steps",
                                       "tally_deposits", "launches", "kernel_ms", "kernel_launches",
                                       "queue_items", "lane_iters", "wave_iters")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
