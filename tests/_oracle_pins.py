"""Pins of the CPU oracle that read its event trace (oracle.run_traced) or call its physics
entry points, written as plain functions of the oracle module so that the same checks run
against the oracle as built (tests/test_oracle_events.py) and against builds with a planted
mistake (tests/test_oracle_mutations.py), which each must fail.

Every check compares with something the oracle does not compute itself: conservation of
energy and momentum, the mathematical form of a distribution (1/k, uniform, isotropic,
Rayleigh), special cases where a formula collapses to a closed value, re-binning of the
recorded deposits, or a quadrature of the cross sections along the recorded tracks."""
from __future__ import annotations

import copy
import ctypes as ct
import math

import numpy as np
from scipy import integrate, stats

from paper_2510_24154_amd import synth

MEC2 = 0.51099895
WCUT, KCUT = 0.200, 0.010
EV = dict(DEPOSIT=0, ESTEP=1, COMPTON=2, PHOTO=3, PAIR=4, ANNIH=5, MOLLER=6, BREMS=7, NULL=8)
P_KS = 1e-3


def _p(T):
    """momentum (MeV/c) of a particle of kinetic energy T and rest energy m c^2 = MEC2"""
    return np.sqrt(T * (T + 2.0 * MEC2))


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _angle(a, b):
    """angle between unit vectors, accurate for small angles"""
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1))


# ---------------------------------------------------------------- workloads
def copper_block(E=6.0, coupled=0):
    """Mono-energetic photons from the point source onto a 3 cm copper block at the isocentre
    (pair production is a quarter of the interactions at 6 MeV)."""
    cfg = synth.coupled_hetero_small()
    cfg["physics"]["coupled"] = coupled
    cfg["source"]["edges"] = np.array([E, E])
    cfg["source"]["weights"] = np.array([1.0])
    cfg["phantom"] = {"kind": "direct", "shape": (1, 1, 1), "spacing": (20.0, 20.0, 3.0),
                      "origin": (-10.0, -10.0, 98.5), "mat": np.array([4], np.uint8),
                      "rho": np.array([8.96])}
    return cfg


def electron_beam(T0, n_list=64, mask=0b111, size=40.0, material=2, rho=1.0):
    """A phase-space list of electrons of kinetic energy T0 at the centre of one large voxel of
    `material` (index into the coupled workload's table), moving along +z."""
    cfg = synth.coupled_hetero_small()
    cfg["physics"]["proc_mask"] = mask
    c = 100.0
    cfg["phantom"] = {"kind": "direct", "shape": (1, 1, 1), "spacing": (size,) * 3,
                      "origin": (-0.5 * size, -0.5 * size, c - 0.5 * size),
                      "mat": np.array([material], np.uint8), "rho": np.array([rho])}
    ps = np.zeros((n_list, 8))
    ps[:, 2] = c
    ps[:, 5] = 1.0
    ps[:, 6] = T0
    ps[:, 7] = 1
    return cfg, ps


def tiny_grid():
    """2 x 2 x 2 voxels (water, lung, bone, air mixed) under the coupled workload's beam, the
    4-layer EPID and a 2 x 2 image of 6 cm pixels."""
    cfg = synth.coupled_hetero_small()
    cfg["phantom"] = {"kind": "direct", "shape": (2, 2, 2), "spacing": (10.0, 10.0, 10.0),
                      "origin": (-10.0, -10.0, 90.0), "mat": np.array([2, 1, 3, 2, 3, 2, 0, 1], np.uint8),
                      "rho": np.array([1.0, 0.3, 1.6, 1.05, 1.85, 0.9, 0.0012, 0.25])}
    cfg["epid"].update(npx_u=2, npx_v=2, pitch_u=6.0, pitch_v=6.0)
    return cfg


def traced(orc, cfg, n, seed=1001, phsp=None, cap=1 << 22):
    return orc.run_traced(cfg, n, seed=seed, cap=cap, phsp=phsp)


# ---------------------------------------------------------------- interaction kinematics
def pin_compton_kinematics(orc):
    """Every Compton event conserves energy (E = E' + T) and momentum: the electron momentum
    E d0 - E' d1 has the magnitude sqrt(T (T + 2 m c^2)) of an electron of kinetic energy T,
    and the electron moves along it.  A wrong scattering angle for the sampled E' breaks
    the magnitude."""
    *_, ev = traced(orc, synth.coupled_hetero_small(), 4000)
    c = ev[ev["kind"] == EV["COMPTON"]]
    assert len(c) > 5000, len(c)
    E, Ep, T = c["E0"], c["E1"], c["Ec"][:, 0]
    assert np.all(np.abs(E - Ep - T) <= 1e-12 * E)
    pe = E[:, None] * c["d0"] - Ep[:, None] * c["d1"]
    pm = np.linalg.norm(pe, axis=1)
    assert np.all(np.abs(pm - _p(T)) <= 1e-8 * _p(T) + 1e-12), np.max(np.abs(pm - _p(T)) / _p(T))
    assert np.all(np.linalg.norm(c["dc"][:, 0] - pe / pm[:, None], axis=1) < 1e-9)
    ph = ev[ev["kind"] == EV["PHOTO"]]
    assert len(ph) > 100
    assert np.array_equal(ph["Ec"][:, 0], ph["E0"]) and np.array_equal(ph["dc"][:, 0], ph["d0"])


def pin_pair_and_annihilation(orc):
    """Pair production: the electron and positron share E - 2 m c^2 with the electron's share
    uniform on (0, 1), both along the photon.  Annihilation at rest: two photons of m c^2,
    back to back, the first isotropic (cos theta uniform on (-1, 1), azimuth uniform)."""
    *_, ev = traced(orc, copper_block(), 12000)
    pr = ev[ev["kind"] == EV["PAIR"]]
    assert len(pr) > 1000, len(pr)
    T = pr["E0"] - 2.0 * MEC2
    assert np.all(np.abs(pr["Ec"][:, 0] + pr["Ec"][:, 1] - T) <= 1e-12 * pr["E0"])
    assert np.array_equal(pr["dc"][:, 0], pr["d0"]) and np.array_equal(pr["dc"][:, 1], pr["d0"])
    assert stats.kstest(pr["Ec"][:, 0] / T, "uniform").pvalue > P_KS
    an = ev[ev["kind"] == EV["ANNIH"]]
    assert len(an) > 1000, len(an)
    assert np.all(an["Ec"] == MEC2)
    a, b = an["dc"][:, 0], an["dc"][:, 1]
    assert np.all(a == -b)
    assert np.all(np.abs(np.linalg.norm(a, axis=1) - 1.0) < 1e-12)
    assert stats.kstest(a[:, 2], stats.uniform(-1.0, 2.0).cdf).pvalue > P_KS
    assert stats.kstest(np.arctan2(a[:, 1], a[:, 0]), stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > P_KS


def pin_moller_and_brems_kinematics(orc):
    """Moller events conserve energy and momentum (p(T) d0 = p(T') d1 + p(W) d_delta, the
    two-body kinematics of electron-electron scattering) with W in [W_c, T/2]; bremsstrahlung
    events take k in [k_c, T] off the electron, which keeps its direction, and emit the photon
    along it."""
    cfg, ps = electron_beam(3.0, mask=0b111 | 16)
    *_, ev = traced(orc, cfg, 6000, phsp=ps)
    m = ev[ev["kind"] == EV["MOLLER"]]
    assert len(m) > 300, len(m)
    T, Tp, W = m["E0"], m["E1"], m["Ec"][:, 0]
    assert np.all(np.abs(T - Tp - W) <= 1e-12 * T)
    assert np.all((W >= WCUT) & (W <= 0.5 * T * (1 + 1e-12)))
    lhs = _p(T)[:, None] * m["d0"]
    rhs = _p(Tp)[:, None] * m["d1"] + _p(W)[:, None] * m["dc"][:, 0]
    assert np.all(np.linalg.norm(lhs - rhs, axis=1) <= 1e-8 * _p(T)), np.max(np.linalg.norm(lhs - rhs, axis=1) / _p(T))
    b = ev[ev["kind"] == EV["BREMS"]]
    assert len(b) > 100, len(b)
    T, Tn, k = b["E0"], b["E1"], b["Ec"][:, 0]
    assert np.all(np.abs(T - Tn - k) <= 1e-12 * T)
    assert np.all((k >= KCUT * (1 - 1e-12)) & (k <= T))
    assert np.array_equal(b["d1"], b["d0"]) and np.array_equal(b["dc"][:, 0], b["d0"])


# ---------------------------------------------------------------- bremsstrahlung
def pin_brems_sampler(orc):
    """The sampler the transport calls draws k from the 1/k law on [k_c, T]: its CDF is
    ln(k / k_c) / ln(T / k_c)."""
    L = orc.lib()
    rng = np.random.default_rng(7)
    for T in (0.3, 2.0, 6.0):
        k = np.array([L.orc_brems_sample(T, KCUT, x) for x in rng.random(40000)])
        assert k.min() >= KCUT * (1 - 1e-12) and k.max() <= T * (1 + 1e-12)
        cdf = lambda x, T=T: np.log(np.clip(x, KCUT, T) / KCUT) / math.log(T / KCUT)
        assert stats.kstest(k, cdf).pvalue > P_KS, T


def pin_brems_energy_balance(orc):
    """The radiative loss is split exactly at k_c: the soft part kept in the restricted loss
    (L_res minus the restricted collision loss) plus the hard part (Sigma_brems times the mean
    k of the sampler, by a midpoint quadrature over its uniform) is the radiative stopping
    power S_rad.  Ties the cross section, the sampler and the soft loss together."""
    L = orc.lib()
    M = 20000
    xi = (np.arange(M) + 0.5) / M
    for m in (synth.WATER, synth.GOS, synth.COPPER):
        mm = orc.material(m)
        for T in (0.3, 1.0, 5.0):
            soft = L.orc_lres(ct.byref(mm), T, WCUT, KCUT) - L.orc_lcol(ct.byref(mm), T, 1, WCUT)
            kbar = np.mean([L.orc_brems_sample(T, KCUT, x) for x in xi])
            hard = L.orc_sigma_brems(ct.byref(mm), T, KCUT) * kbar
            assert abs(soft + hard - L.orc_srad(ct.byref(mm), T)) <= 1e-6 * L.orc_srad(ct.byref(mm), T), (m["name"], T)


def pin_srad_magnitude(orc):
    """Water's radiative stopping power has the textbook magnitude (ESTAR-like values: about
    0.013 MeV cm^2/g at 1 MeV and about 0.10 at 6 MeV).  The S_rad/S_col = Z_eff T / 800 MeV
    rule is good to a few tens of percent, so the band is +-35%; a dropped Z_eff (x 6.6) or
    a dropped factor T fails it."""
    L = orc.lib()
    w = orc.material(synth.WATER)
    assert 0.65 * 0.013 < L.orc_srad(ct.byref(w), 1.0) < 1.35 * 0.013
    assert 0.65 * 0.10 < L.orc_srad(ct.byref(w), 6.0) < 1.35 * 0.10


# ---------------------------------------------------------------- multiple scattering
def pin_highland_special_cases(orc):
    """Highland's width theta0 = 13.6 MeV / (beta c p) sqrt(x/X0) [1 + 0.038 ln(x / (X0 beta^2))]
    (PDG, unit charge) collapses at x = X0 beta^2 to 13.6 MeV / (c p), and at x = e X0 beta^2
    and x = X0 beta^2 / e to 13.6 sqrt(e) 1.038 / (c p) and 13.6 (1 - 0.038) / (sqrt(e) c p):
    the constant, the momentum, the square root and the 0.038 ln term each change them."""
    L = orc.lib()
    for T in (0.25, 1.0, 3.0, 12.0):
        pc = math.sqrt(T * (T + 2 * MEC2))
        b2 = pc * pc / (T + MEC2) ** 2
        for X0 in (36.08, 1.436, 6.5):
            x = X0 * b2
            assert L.orc_highland(T, x, X0) == _approx(13.6 / pc)
            assert L.orc_highland(T, math.e * x, X0) == _approx(13.6 * math.sqrt(math.e) * 1.038 / pc)
            assert L.orc_highland(T, x / math.e, X0) == _approx(13.6 * (1 - 0.038) / (math.sqrt(math.e) * pc))


def _approx(v, rel=1e-12):
    import pytest
    return pytest.approx(v, rel=rel)


def pin_msc_rayleigh_and_hinge(orc):
    """With hard events off, the first step of a 2 MeV electron in a large water voxel is the
    10% energy-loss step; its deflection is the random-hinge angle, Rayleigh-distributed with
    the Highland width of that step (PDG), and the hinge point, where the continuous loss is
    left, lies on the initial direction at a fraction of the step uniform on (0, 1)."""
    cfg, ps = electron_beam(2.0, mask=0b111 | 8)
    *_, ev = traced(orc, cfg, 5000, phsp=ps)
    st = ev[ev["kind"] == EV["ESTEP"]]
    first = st[np.r_[True, st["hist"][1:] != st["hist"][:-1]]]
    assert len(first) == 5000
    assert np.all(first["E0"] == 2.0)
    x = first["aux"][:, 1]
    assert np.ptp(x) <= 1e-12 * x[0]                 # the same 10% energy-loss step every time
    th0 = orc.lib().orc_highland(2.0, float(x[0]), float(first["Ec"][0, 0]))
    th = _angle(first["d0"], first["d1"])
    assert stats.kstest(th, stats.rayleigh(scale=th0).cdf).pvalue > P_KS
    rel = first["dc"][:, 0] - first["pos"]
    s = first["aux"][:, 0]
    along = np.sum(rel * first["d0"], axis=1)
    assert np.all(np.linalg.norm(rel - along[:, None] * first["d0"], axis=1) <= 1e-9 * s)
    assert stats.kstest(along / s, "uniform").pvalue > P_KS


# ---------------------------------------------------------------- hard-event rate
def sigma_hard(orc, mm, T):
    L = orc.lib()
    return L.orc_sigma_moller(ct.byref(mm), T, WCUT) + L.orc_sigma_brems(ct.byref(mm), T, KCUT)


def pin_sigma_hard_majorant(orc):
    """Sigma_hard(T) falls and then rises with T over the transported energies (one minimum),
    so on any step's interval [0.9 T0, T0] it is bounded by the larger end value, which is the
    majorant the hard-event distance is drawn against."""
    L = orc.lib()
    T = np.geomspace(0.18, 60.0, 3000)
    for m in (synth.WATER, synth.BONE, synth.COPPER, synth.GOS, synth.GLASS, synth.PET, synth.AIR):
        mm = orc.material(m)
        sh = np.array([sigma_hard(orc, mm, t) for t in T])
        sign = np.sign(np.diff(sh))
        sign = sign[sign != 0]
        assert np.count_nonzero(np.diff(sign) != 0) <= 1 and sign[-1] > 0, m["name"]
        for T0 in (0.21, 0.39, 0.42, 0.44, 0.9, 4.0):
            grid = np.linspace(0.9 * T0, T0, 200)
            assert L.orc_sigma_hard_max(ct.byref(mm), T0, WCUT, KCUT) >= max(sigma_hard(orc, mm, t) for t in grid)


def pin_hard_event_rate(orc, T0=0.7, n=20000):
    """Electrons of 0.7 MeV in Gd2O2S (multiple scattering off): the numbers of real Moller
    and bremsstrahlung events each equal the integral of their cross section along the
    recorded tracks, which in energy is int Sigma(T) / L_res(T) dT over every step (Poisson
    z; the integrals from cumulative tables of per-interval quadratures).  The distance to a
    candidate event is drawn against the step's largest hard cross section and a candidate is
    kept with probability Sigma_hard(T1) over it (thinning), which makes these rates exact."""
    cfg, ps = electron_beam(T0, mask=0b111 | 16, material=6, rho=7.44)
    *_, ev = traced(orc, cfg, n, phsp=ps, cap=1 << 23)
    L = orc.lib()
    mm = orc.material(synth.GOS)
    st = ev[(ev["kind"] == EV["ESTEP"]) & (ev["aux"][:, 1] > 0)]
    grid = np.unique(np.concatenate([np.linspace(0.15, T0 * 1.001, 1500), [2 * WCUT]]))
    for kind, sig in ((EV["MOLLER"], lambda t: L.orc_sigma_moller(ct.byref(mm), t, WCUT)),
                      (EV["BREMS"], lambda t: L.orc_sigma_brems(ct.byref(mm), t, KCUT))):
        f = lambda t: sig(t) / L.orc_lres(ct.byref(mm), t, WCUT, KCUT)
        F = np.concatenate([[0.0], np.cumsum([integrate.quad(f, lo, hi, epsrel=1e-10)[0]
                                              for lo, hi in zip(grid[:-1], grid[1:])])])
        expect = float(np.sum(np.interp(st["E0"], grid, F) - np.interp(st["E1"], grid, F)))
        seen = int(np.count_nonzero(ev["kind"] == kind))
        assert expect > 400, expect
        z = (seen - expect) / math.sqrt(expect)
        assert abs(z) < 4, (kind, seen, expect, z)


# ---------------------------------------------------------------- tally (G-BF)
def pin_tiny_grid_rebinning(orc):
    """Brute force on a 2 x 2 x 2 phantom and a 2 x 2 image: every recorded deposit that lies in
    the scoring layer within the image is tallied to the pixel its position falls in, and only
    those; each deposit's EPID layer is the one whose planes hold its position; and adding the
    recorded deposits history by history reproduces the oracle's sum and sum of squares
    exactly."""
    cfg = tiny_grid()
    _, _, s, s2, c, ev = traced(orc, cfg, 10000)
    E = cfg["epid"]
    zl = E["front_z"] + np.concatenate([[0.0], np.cumsum([l["t"] for l in E["layers"]])])
    hx, hy = 0.5 * E["npx_u"] * E["pitch_u"], 0.5 * E["npx_v"] * E["pitch_v"]
    d = ev[ev["kind"] == EV["DEPOSIT"]]
    ep = d[d["region"] == 1]
    assert len(ep) > 1000
    lay = np.searchsorted(zl, ep["pos"][:, 2], side="right") - 1
    assert np.array_equal(ep["layer"], lay)
    fu = np.floor((ep["pos"][:, 0] + hx) / E["pitch_u"])
    fv = np.floor((ep["pos"][:, 1] + hy) / E["pitch_v"])
    inside = (fu >= 0) & (fu < E["npx_u"]) & (fv >= 0) & (fv < E["npx_v"])
    want = np.where((lay == E["scoring"]) & inside & (ep["E0"] > 0), fv * E["npx_u"] + fu, -1).astype(np.int64)
    assert np.array_equal(ep["pixel"].astype(np.int64), want)
    assert np.all(d["pixel"][d["region"] != 1] == -1)
    tal = d[d["pixel"] >= 0]
    assert len(tal) == c["n_tally_deposits"] > 100
    rs, rs2 = np.zeros_like(s), np.zeros_like(s2)
    for h in np.unique(tal["hist"]):
        acc = {}
        for e in tal[tal["hist"] == h]:
            acc[int(e["pixel"])] = acc.get(int(e["pixel"]), 0.0) + float(e["E0"])
        for p, v in acc.items():
            rs[p] += v
            rs2[p] += v * v
    assert np.array_equal(rs, s) and np.array_equal(rs2, s2)


def pin_step_floor_bias(orc, n=640_000, parts=16, threads=8):
    """What a floor on boundary-limited electron steps would do.  The reading has none: a step
    never carries a cell's medium across a face.  A floor of 5% of the cell's smallest side
    (which an earlier reading used to avoid strings of very short steps along faces) lets a
    step run up to that far into the next cell with the wrong stopping power.  On the coupled
    workload the floor-on and floor-off images pass the z-gate on 4 x 4 bins, and their
    scoring-layer totals, from `parts` independent sub-runs each, differ by less than 3.5
    standard deviations (the floor lowers the phosphor total by about 2%, within about 1.5
    standard deviations at 4e6 histories).  Returns the gate, the relative total difference
    and its standard deviation."""
    from tests._stats import z_gate
    a = synth.coupled_hetero_small()
    a["physics"]["step_floor"] = 0.05
    b = copy.deepcopy(a)
    b["physics"]["step_floor"] = 0.0
    m = n // parts
    out = []
    for cfg, seed in ((a, 11), (b, 12)):
        img, var, tot = 0.0, 0.0, []
        for i in range(parts):
            mi, vi, *_ = orc.run(cfg, m, seed=seed, first=i * m, threads=threads)
            img = img + mi / parts
            var = var + vi / parts ** 2
            tot.append(mi.sum())
        out.append((img, var, np.array(tot)))
    (ma, va, ta), (mb, vb, tb) = out
    g = z_gate(ma, va, mb, vb, thr=0.10, k=4)
    assert g["ok"], g
    d = ta.mean() - tb.mean()
    sd = math.sqrt(ta.var(ddof=1) / parts + tb.var(ddof=1) / parts)
    assert abs(d) < 3.5 * sd, (d, sd)
    return g, d / ta.mean(), sd / ta.mean()
