"""Statistical comparison tools for Monte Carlo images (test-side only).

z_gate: per-pixel standard scores of the difference of two independent MC
estimates, judged as a population (pass fraction, mean, spread) because a
literal "every pixel within 2 sigma" rejects ~4.6% of correct pixels.

gamma_pass: global gamma index (Low et al. 1998), dose criterion relative to
the reference maximum, low-dose threshold on the reference, distance search on
a sub-pixel grid of the evaluated image (Sec. 2.3.3 names global 3%/3 mm,
3%/2 mm and 2%/2 mm with a 10% threshold).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage


def rebin(a, k):
    if k == 1:
        return a
    v, u = a.shape
    return a[: v - v % k, : u - u % k].reshape(v // k, k, u // k, k).sum(axis=(1, 3))


def z_gate(d1, v1, d2, v2, thr=0.10, k=1):
    """d1/v1: first image and the variance of its mean; d2/v2: reference image.
    Images may be k x k binned first (sums of means, sums of variances)."""
    d1, v1, d2, v2 = (rebin(np.asarray(x, dtype=np.float64), k) for x in (d1, v1, d2, v2))
    sel = d2 >= thr * d2.max()
    s = np.sqrt(v1[sel] + v2[sel])
    ok = s > 0
    z = (d1[sel][ok] - d2[sel][ok]) / s[ok]
    n = z.size
    frac = float(np.mean(np.abs(z) <= 2.0)) if n else 0.0
    need = 0.9545 - 3.0 * math.sqrt(0.0455 * 0.9545 / max(n, 1))
    mz, sz = (float(z.mean()), float(z.std(ddof=1))) if n > 1 else (0.0, 0.0)
    res = {"n": int(n), "frac_within_2": frac, "frac_needed": need, "mean_z": mz, "sd_z": sz,
           "mean_bound": 3.0 / math.sqrt(max(n, 1))}
    res["ok"] = bool(n > 30 and frac >= need and abs(mz) <= res["mean_bound"] and 0.9 <= sz <= 1.1)
    return res


def gamma_map(ref, evl, pitch, dd=0.02, dta=0.2, pitch_v=None):
    """Per-pixel global gamma of the evaluated image against the reference.

    ref, evl: 2D images on the same grid; pitch in cm (u = fast axis), dta in cm,
    dd as a fraction of max(ref).  The evaluated image is searched within a radius
    of dta on a grid of spacing <= dta/3 by bilinear interpolation."""
    ref = np.asarray(ref, dtype=np.float64)
    evl = np.asarray(evl, dtype=np.float64)
    pu, pv = pitch, (pitch if pitch_v is None else pitch_v)
    dcrit = dd * ref.max()
    ku = max(1, math.ceil(pu / (dta / 3.0)))
    kv = max(1, math.ceil(pv / (dta / 3.0)))
    best = np.full(ref.shape, np.inf)
    nu, nv = int(math.floor(dta / (pu / ku))), int(math.floor(dta / (pv / kv)))
    for iv in range(-nv, nv + 1):
        for iu in range(-nu, nu + 1):
            dx, dy = iu * pu / ku, iv * pv / kv
            r2 = (dx * dx + dy * dy) / (dta * dta)
            if r2 > 1.0:
                continue
            sh = ndimage.shift(evl, (-iv / kv, -iu / ku), order=1, mode="nearest")
            g2 = r2 + ((sh - ref) / dcrit) ** 2
            np.minimum(best, g2, out=best)
    return np.sqrt(best)


def gamma_pass(ref, evl, pitch, dd=0.02, dta=0.2, thr=0.10, pitch_v=None):
    """Fraction of reference pixels (D >= thr * max) with gamma <= 1 (see gamma_map)."""
    ref = np.asarray(ref, dtype=np.float64)
    sel = ref >= thr * ref.max()
    g = gamma_map(ref, evl, pitch, dd=dd, dta=dta, pitch_v=pitch_v)
    return float(np.mean(g[sel] <= 1.0))


def sigma_bar(mean, var, thr=0.5):
    """Mean relative standard deviation over pixels with D >= thr * max (TG-105 style)."""
    sel = mean >= thr * mean.max()
    return float(np.mean(np.sqrt(var[sel]) / mean[sel]))
