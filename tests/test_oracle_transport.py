"""Pins of the oracle's transport against closed forms it does not compute itself:
narrow-beam transmission exp(-sum mu rho l), pixel-resolved absorption images with
no scatter, the divergent-beam geometry, first-collision KERMA, the per-history
energy ledger, mirror symmetry, source sampling and CSDA track length.  CPU only."""
import copy
import ctypes as ct
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2510_24154_amd import synth

MEC2 = 0.51099895
THREADS = 8


def mu(orc, m, E, mask=0b111):
    out = np.zeros(4)
    orc.lib().orc_photon_mu(ct.byref(orc.material(m)), E, out.ctypes.data)
    return sum(out[1 + i] for i in range(3) if mask >> i & 1)


def binom_z(k, n, p):
    return (k - n * p) / math.sqrt(n * p * (1 - p))


def test_transmission_water_box(orc):
    """Unscattered 2 MeV primaries behind 20 cm of water: exp(-20 mu_w)."""
    cfg = synth.kerma_water()
    n = 300_000
    _, _, _, _, c = orc.run(cfg, n, threads=THREADS)
    p = math.exp(-20.0 * mu(orc, synth.WATER, 2.0, 0b011))
    assert abs(binom_z(c["unscattered_at_epid"], n, p)) < 4


def _slab_phantom(cfg, slabs, nxy=4):
    """Replace the phantom by slabs along z: list of (material index, density, n_voxels)."""
    nz = sum(s[2] for s in slabs)
    mats = np.concatenate([np.full(s[2], s[0], np.uint8) for s in slabs])
    rhos = np.concatenate([np.full(s[2], s[1], np.float64) for s in slabs])
    P = cfg["phantom"]
    sp = P["spacing"]
    cfg["phantom"] = {"kind": "direct", "shape": (nxy, nxy, nz), "spacing": (sp[0] * 25, sp[1] * 25, sp[2]),
                      "origin": (-0.5 * nxy * sp[0] * 25, -0.5 * nxy * sp[1] * 25, 0.0),
                      "mat": np.repeat(mats, nxy * nxy), "rho": np.repeat(rhos, nxy * nxy)}
    return cfg


def test_transmission_heterogeneous_slabs(orc):
    cfg = synth.coupled_hetero_small()
    cfg["physics"]["coupled"] = 0
    cfg["source"] = synth.kerma_water()["source"]
    cfg["source"]["edges"] = np.array([1.25, 1.25])
    slabs = [(2, 1.0, 10), (3, 1.6, 7), (1, 0.3, 20), (3, 1.85, 3), (0, 0.0012, 5), (2, 1.0, 15)]
    cfg = _slab_phantom(cfg, slabs)
    dz = cfg["phantom"]["spacing"][2]
    mats = cfg["materials"]
    tau = sum(mu(orc, mats[m], 1.25) * rho * k * dz for m, rho, k in slabs)
    n = 200_000
    _, _, _, _, c = orc.run(cfg, n, threads=THREADS)
    assert abs(binom_z(c["unscattered_at_epid"], n, math.exp(-tau))) < 4


def _absorption_only(cfg, E):
    cfg["physics"] = {"coupled": 0, "proc_mask": 0b010, "pcut": 0.01, "ecut": 0.2}
    cfg["source"]["edges"] = np.array([E, E])
    cfg["source"]["weights"] = np.array([1.0])
    return cfg


def test_pixel_resolved_absorption_parallel(orc):
    """Photoelectric-only parallel beam through columns of different density onto a lone
    phosphor layer: every pixel's expected deposit is E * (pixel area / beam area) *
    exp(-mu rho_col L) * (1 - exp(-mu_g rho_g t_g)).  Column densities differ along x and
    y, so a transposed or mirrored index fails."""
    E = 0.03
    cfg = _absorption_only(synth.kerma_water(), E)
    nc = 4
    rng = np.random.default_rng(7)
    col = rng.uniform(0.1, 1.0, (nc, nc))             # [iy][ix]
    Lz = 4.0
    cfg["phantom"] = {"kind": "direct", "shape": (nc, nc, 4), "spacing": (2.5, 2.5, Lz / 4),
                      "origin": (-5.0, -5.0, 0.0), "mat": np.zeros(nc * nc * 4, np.uint8),
                      "rho": np.tile(col.reshape(-1), 4).astype(np.float64)}
    cfg["epid"] = {"layers": [{"mat": 2, "t": 0.003, "rho": 7.44}], "scoring": 0, "front_z": 20.0,
                   "npx_u": 16, "npx_v": 16, "pitch_u": 0.625, "pitch_v": 0.625}
    n = 400_000
    mean, var, _, _, c = orc.run(cfg, n, threads=THREADS)
    mw, mg = mu(orc, synth.WATER, E, 2), mu(orc, synth.GOS, E, 2)
    absorb = 1 - math.exp(-mg * 7.44 * 0.003)
    # pixel (v, u) -> column (v // 4, u // 4)
    expect = np.zeros((16, 16))
    for v in range(16):
        for u in range(16):
            expect[v, u] = E * (0.625 ** 2 / 100.0) * math.exp(-mw * col[v // 4, u // 4] * Lz) * absorb
    # per pixel the deposit count is binomial: var of the mean = E^2 p (1-p) / n
    p = expect / E
    z = (mean - expect) / np.sqrt(E * E * p * (1 - p) / n)
    assert np.all(np.abs(z) < 5), np.abs(z).max()
    assert abs(z.mean()) < 3 / 16
    assert 0.8 < z.std() < 1.2


def test_divergent_geometry_absorption(orc):
    """Point source, photoelectric only, homogeneous water slab: photons per unit area at
    the phosphor follow the magnification SID/SAD, and each pixel sees exp(-mu rho t/cos)."""
    E = 0.1
    cfg = _absorption_only(synth.coupled_hetero_small(), E)
    t = 10.0
    cfg["phantom"] = {"kind": "direct", "shape": (8, 8, 4), "spacing": (6.0, 6.0, t / 4),
                      "origin": (-24.0, -24.0, 95.0), "mat": np.full(256, 2, np.uint8),
                      "rho": np.ones(256)}
    cfg["epid"] = {"layers": [{"mat": 6, "t": 0.002, "rho": 7.44}], "scoring": 0, "front_z": 150.0,
                   "npx_u": 24, "npx_v": 24, "pitch_u": 1.0, "pitch_v": 1.0}
    n = 400_000
    mean, var, _, _, _ = orc.run(cfg, n, threads=THREADS)
    mw, mg = mu(orc, synth.WATER, E, 2), mu(orc, synth.GOS, E, 2)
    M = 150.0 / 100.0
    fluence = 1.0 / (100.0 * M * M)                    # per cm^2 per history at the EPID plane
    z = []
    for v in range(24):
        for u in range(24):
            x, y = -12 + u + 0.5, -12 + v + 0.5
            if abs(x) + 0.5 > 5 * M or abs(y) + 0.5 > 5 * M:     # only pixels fully inside the field
                if abs(x) - 0.5 > 5 * M or abs(y) - 0.5 > 5 * M:
                    assert mean[v, u] == 0.0
                continue
            cosg = 150.0 / math.sqrt(x * x + y * y + 150.0 ** 2)
            p = fluence * math.exp(-mw * t / cosg) * (1 - math.exp(-mg * 7.44 * 0.002 / cosg))
            z.append((mean[v, u] - E * p) / math.sqrt(E * E * p * (1 - p) / n))
    z = np.array(z)
    assert z.size == 14 * 14
    assert np.all(np.abs(z) < 5) and abs(z.mean()) < 3 / 14 and 0.8 < z.std() < 1.2


def kn_mean_transfer(E):
    k = E / MEC2

    def f(c):
        P = 1.0 / (1.0 + k * (1.0 - c))
        return P * P * (P + 1.0 / P - (1.0 - c * c))
    tot = integrate.quad(f, -1, 1, points=[0.9, 0.99], epsrel=1e-12)[0]
    return integrate.quad(lambda c: f(c) * (1 - 1 / (1 + k * (1 - c))), -1, 1, points=[0.9, 0.99],
                          epsrel=1e-12)[0] / tot


def test_first_collision_kerma(orc):
    """Parallel 2 MeV beam through an empty phantom onto Cu + phosphor: first collisions in
    the phosphor per photon = exp(-mu_cu t_cu)(1 - exp(-mu_g t_g)); energy released per
    collision = (mu_C <T> + tau E) / mu with <T> the KN mean transfer."""
    E = 2.0
    cfg = synth.kerma_water(nvox=10)
    cfg["phantom"]["rho"] = np.zeros(1000, np.float32)
    n = 1_000_000
    _, _, _, _, c = orc.run(cfg, n, threads=THREADS)
    L = orc.lib()
    out = np.zeros(4)
    L.orc_photon_mu(ct.byref(orc.material(synth.COPPER)), E, out.ctypes.data)
    mcu = (out[1] + out[2]) * 8.96
    L.orc_photon_mu(ct.byref(orc.material(synth.GOS)), E, out.ctypes.data)
    mc, tp, mg = out[1] * 7.44, out[2] * 7.44, (out[1] + out[2]) * 7.44
    pint = math.exp(-mcu * 0.2) * (1 - math.exp(-mg * 0.03))
    assert abs(binom_z(c["n_first_collision"], n, pint)) < 4
    per = (mc * kn_mean_transfer(E) * E + tp * E) / mg
    # mean released energy per first collision; its spread is bounded by E, use the sample size
    k = c["n_first_collision"]
    assert abs(c["e_first_collision"] / k - per) < 4 * 0.6 * E / math.sqrt(k)


@pytest.mark.parametrize("factory,n", [(synth.kerma_water, 50_000), (synth.coupled_hetero_small, 20_000)])
def test_energy_ledger(orc, factory, n):
    """Per history: incident = deposited + escaped + (pair rest energy not annihilated)."""
    _, _, _, _, c = orc.run(factory(), n, threads=THREADS)
    assert c["max_ledger_resid"] < 1e-9
    tot = c["e_dep_phantom"] + c["e_dep_epid"] + c["e_dep_other"] + c["e_escaped"] + c["e_rest_balance"]
    assert tot == pytest.approx(c["e_in"], rel=1e-12)


def test_mirror_symmetry_coupled(orc):
    """Water-only phantom, symmetric field and image: D(x, y) and D(-x, y), D(x, -y) agree."""
    cfg = synth.coupled_hetero_small()
    cfg["phantom"]["hu"] = np.zeros_like(cfg["phantom"]["hu"])
    n = 60_000
    mean, var, _, _, _ = orc.run(cfg, n, threads=THREADS)
    from tests._stats import rebin
    d, v = rebin(mean, 8), rebin(var, 8)
    for axis in (0, 1):
        df = d - np.flip(d, axis)
        vf = v + np.flip(v, axis)
        sel = (d > 0.1 * d.max()) & (vf > 0)
        z = df[sel] / np.sqrt(vf[sel])
        # each pair appears twice (z and -z): use one of each pair
        z = z[: z.size // 2]
        assert np.all(np.abs(z) < 5) and abs(z.mean()) < 4 / math.sqrt(z.size)


def test_split_ranges_sum_to_whole(orc):
    """Histories are keyed by id: disjoint ranges add up to the whole run (up to summation order)."""
    cfg = synth.coupled_hetero_small()
    P = orc.Prepared(cfg, 99)
    _, _, s, s2, c = orc.run(cfg, 4000, prepared=P, threads=1)
    _, _, sa, s2a, ca = orc.run(cfg, 1500, prepared=P, threads=1)
    _, _, sb, s2b, cb = orc.run(cfg, 2500, first=1500, prepared=P, threads=1)
    np.testing.assert_allclose(sa + sb, s, rtol=1e-12, atol=0)
    np.testing.assert_allclose(s2a + s2b, s2, rtol=1e-12, atol=0)
    assert ca["n_compton"] + cb["n_compton"] == c["n_compton"]


def test_source_spectrum_and_aperture(orc):
    cfg = synth.imrt_field(total=300_000_000)
    ap = cfg["source"]["aperture"]
    # histories of segment 3
    first = int(ap["counts"][:3].sum())
    hs = np.arange(first, first + 40_000)
    src = orc.source(cfg, hs)
    E = src[:, 6]
    edges, w = cfg["source"]["edges"], cfg["source"]["weights"]
    obs, _ = np.histogram(E, edges)
    exp = w / w.sum() * len(hs)
    keep = exp > 5
    assert stats.chi2.sf(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]), keep.sum() - 1) > 1e-3
    # directions from the point source reach the isocentre plane inside segment 3's aperture
    t = 100.0 / src[:, 5]
    x, y = src[:, 3] * t, src[:, 4] * t
    k = np.floor((y - ap["y0"]) / ap["leaf_w"]).astype(int)
    a, b = ap["a"][3][k], ap["b"][3][k]
    assert np.all((x >= a - 1e-9) & (x <= b + 1e-9))
    # leaf pairs are chosen in proportion to their open width
    width = ap["b"][3] - ap["a"][3]
    obs = np.bincount(k, minlength=ap["n_pairs"])
    exp = width / width.sum() * len(hs)
    keep = exp > 5
    assert stats.chi2.sf(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]), keep.sum() - 1) > 1e-3
    # uniform along x within the pair: position within the open interval is U(0, 1)
    f = (x - a) / np.maximum(b - a, 1e-12)
    assert stats.kstest(f[width[k] > 0.5], "uniform").pvalue > 1e-3


def test_csda_track_length_bounds(orc):
    """Hard events and multiple scattering off: a 2 MeV electron travels
    (R(T0) - R(T_end)) / rho with T_end in [0.9 Tcut, Tcut), deposits all its energy."""
    cfg = synth.kerma_water(nvox=10)
    cfg["physics"] = {"coupled": 1, "proc_mask": 0b11111, "pcut": 0.01, "ecut": 0.2}
    ph = np.array([[0.3, -0.2, 5.0, 0.0, 0.0, 1.0, 2.0, 1.0]])
    n = 50
    _, _, _, _, c = orc.run(cfg, n, phsp=ph, threads=1)
    L = orc.lib()
    w = orc.material(synth.WATER)
    lo = L.orc_range_diff(ct.byref(w), 0.2, 2.0, 0.2, 0.01)
    hi = L.orc_range_diff(ct.byref(w), 0.18, 2.0, 0.2, 0.01)
    per = c["e_track"] / n
    assert lo <= per <= hi
    assert c["e_dep_phantom"] == pytest.approx(2.0 * n, rel=1e-12)
    assert c["n_moller"] == 0 and c["n_brems"] == 0
