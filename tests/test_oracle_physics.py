"""Pins of the oracle's physics functions against mathematics that does not go
through the oracle's own formulas: published known-answer vectors, limits,
quadratures of differential cross sections written in another parametrisation,
invariants, and textbook magnitudes.  CPU only."""
import ctypes as ct
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2510_24154_amd import synth

MEC2 = 0.51099895
RE = 2.8179403262e-13
NA = 6.02214076e23


def _mat(orc, m):
    return orc.material(m)


# ---------------------------------------------------------------- Philox
KAT = [  # Random123 known-answer vectors for Philox4x32-10: counter, key -> output
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


def _philox(orc, c, k):
    c = np.array(c, dtype=np.uint32)
    k = np.array(k, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    orc.lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return [int(x) for x in o]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(orc, ctr, key, out):
    assert _philox(orc, ctr, key) == out


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned s = 12345u;
  for (int i = 0; i < 64; ++i) {
    unsigned v[6];
    for (int j = 0; j < 6; ++j) { s = s * 1664525u + 1013904223u; v[j] = s; }
    v[1] &= 0x3fffffffu;   /* keep 4 * offset inside 64 bits */
    rocrand_state_philox4x32_10 st;
    unsigned long long key = ((unsigned long long)v[5] << 32) | v[4];
    unsigned long long sub = ((unsigned long long)v[3] << 32) | v[2];
    unsigned long long off = 4ull * (((unsigned long long)v[1] << 32) | v[0]);
    rocrand_init(key, sub, off, &st);
    unsigned r0 = rocrand(&st), r1 = rocrand(&st), r2 = rocrand(&st), r3 = rocrand(&st);
    printf("%u %u %u %u %u %u %u %u %u %u\n", v[0], v[1], v[2], v[3], v[4], v[5], r0, r1, r2, r3);
  }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(orc):
    """rocRAND's Philox4x32-10 (run through its public API, not copied) on 64
    pseudo-random counters and keys: counter = (offset/4, subsequence), key = seed."""
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "p.cpp"), os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROBE)
        r = subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-o", exe, src],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("rocRAND probe did not compile: " + r.stderr[-300:])
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    n = 0
    for ln in lines:
        if not ln.strip():
            continue
        v = [int(x) for x in ln.split()]
        assert _philox(orc, v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 64


# ---------------------------------------------------------------- Klein-Nishina
def kn_dsdomega(E, ct_):
    """Klein-Nishina differential cross section per electron, cm^2/sr, in the angle form."""
    P = 1.0 / (1.0 + E / MEC2 * (1.0 - ct_))
    return 0.5 * RE * RE * P * P * (P + 1.0 / P - (1.0 - ct_ * ct_))


def kn_sigma_ref(E):
    """Total KN cross section per electron by a 30-digit quadrature of the angular form."""
    import mpmath as mp
    mp.mp.dps = 30
    k = mp.mpf(E) / mp.mpf(MEC2)

    def f(c):
        P = 1 / (1 + k * (1 - c))
        return P * P * (P + 1 / P - (1 - c * c))

    return float(mp.pi * mp.mpf(RE) ** 2 * mp.quad(f, [-1, 0, 0.9, 0.99, 0.999, 1]))


@pytest.mark.parametrize("E", [0.01, 0.1, 0.511, 2.0, 6.0, 50.0])
def test_kn_total_equals_angular_integral(orc, E):
    assert orc.lib().orc_sigma_kn(E) == pytest.approx(kn_sigma_ref(E), rel=1e-12)


def test_kn_limits(orc):
    sT = 8 * math.pi / 3 * RE * RE
    k = 1e-4 / MEC2
    # low-energy series sigma_T (1 - 2k + 26/5 k^2)
    assert orc.lib().orc_sigma_kn(1e-4) == pytest.approx(sT * (1 - 2 * k + 5.2 * k * k), rel=1e-9)
    E = 5000.0
    k = E / MEC2
    asym = math.pi * RE * RE / k * (math.log(2 * k) + 0.5)
    assert orc.lib().orc_sigma_kn(E) == pytest.approx(asym, rel=2e-3)


@pytest.mark.parametrize("E", [0.05, 0.5, 2.0, 6.0])
def test_kn_cdf_matches_angular_integral(orc, E):
    """CDF in eps against a 30-digit quadrature of the angular form over cos(theta)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    k = mp.mpf(E) / mp.mpf(MEC2)

    def f(c):
        P = 1 / (1 + k * (1 - c))
        return P * P * (P + 1 / P - (1 - c * c))

    brk = [-1, 0, 0.9, 0.99, 0.999, 1]
    tot = mp.quad(f, brk)
    for eps in np.linspace(1 / (1 + 2 * float(k)), 1.0, 7)[1:-1]:
        c_lim = 1 - (1 / mp.mpf(eps) - 1) / k          # eps <= e  <=>  cos(theta) <= c_lim
        part = mp.quad(f, [b for b in brk if b < c_lim] + [c_lim])
        assert orc.lib().orc_kn_cdf(E, eps) == pytest.approx(float(part / tot), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("E", [0.1, 0.5, 2.0, 6.0])
def test_kn_sampler_chi2(orc, E):
    """Inverse-CDF sampler against the angular KN density binned in cos(theta)."""
    rng = np.random.default_rng(int(E * 1000))
    n = 100_000
    k = E / MEC2
    L = orc.lib()
    eps = np.array([L.orc_kn_sample(E, x) for x in rng.random(n)])
    cth = 1.0 - (1.0 / eps - 1.0) / k
    edges = np.linspace(-1, 1, 41)
    obs, _ = np.histogram(cth, edges)
    tot = integrate.quad(lambda c: kn_dsdomega(E, c), -1, 1, epsrel=1e-12)[0]
    exp = np.array([integrate.quad(lambda c: kn_dsdomega(E, c), a, b, epsrel=1e-12)[0]
                    for a, b in zip(edges[:-1], edges[1:])]) / tot * n
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    p = stats.chi2.sf(chi2, keep.sum() - 1)
    assert p > 1e-3, (chi2, p)
    # mean energy transfer <T>/E against quadrature
    mt = integrate.quad(lambda c: kn_dsdomega(E, c) * (1 - 1 / (1 + k * (1 - c))), -1, 1, epsrel=1e-12)[0] / tot
    se = np.std(1 - eps) / math.sqrt(n)
    assert abs(np.mean(1 - eps) - mt) < 4 * se


# ---------------------------------------------------------------- photon attenuation
def _mu(orc, m, E):
    out = np.zeros(4)
    orc.lib().orc_photon_mu(ct.byref(_mat(orc, m)), E, out.ctypes.data)
    return out


def test_bragg_additivity(orc):
    """A compound's mu/rho is the mass-fraction weighted sum of its elements'."""
    for m in (synth.WATER, synth.BONE, synth.GOS, synth.PET):
        for E in (0.02, 0.3, 1.5, 5.0):
            tot = np.zeros(4)
            for z, a, w in zip(m["Z"], m["A"], m["w"]):
                tot += w * _mu(orc, {"Z": [z], "A": [a], "w": [1.0], "I_eV": 1.0}, E)
            np.testing.assert_allclose(_mu(orc, m, E), tot, rtol=1e-12)


def test_compton_is_electron_density_times_kn(orc):
    ne = NA * sum(w * z / a for z, a, w in zip(synth.WATER["Z"], synth.WATER["A"], synth.WATER["w"]))
    assert ne == pytest.approx(NA * 10 / 18.015, rel=1e-4)   # 10 electrons per 18.015 g
    for E in (0.05, 1.0, 4.0):
        assert _mu(orc, synth.WATER, E)[1] == pytest.approx(ne * kn_sigma_ref(E), rel=1e-12)


def test_photoelectric_scaling(orc):
    cu = {"Z": [29], "A": [63.546], "w": [1.0], "I_eV": 1}
    o = {"Z": [8], "A": [15.999], "w": [1.0], "I_eV": 1}
    for E in (0.02, 0.2, 2.0):
        assert _mu(orc, cu, 2 * E)[2] == pytest.approx(_mu(orc, cu, E)[2] / 8, rel=1e-12)   # E^-3
        ratio = _mu(orc, cu, E)[2] / _mu(orc, o, E)[2]
        assert ratio == pytest.approx((29 / 8) ** 4 * 15.999 / 63.546, rel=1e-12)       # Z^4 per atom


def test_water_photo_compton_crossover(orc):
    """Calibration reading: the photoelectric constant puts water's photoelectric and
    Compton attenuation equal near 27 keV (textbook crossover 25-30 keV)."""
    from scipy.optimize import brentq
    e = brentq(lambda E: _mu(orc, synth.WATER, E)[2] - _mu(orc, synth.WATER, E)[1], 0.015, 0.06)
    assert 0.025 < e < 0.030


def test_pair_threshold_and_magnitude(orc):
    w = synth.WATER
    assert _mu(orc, w, 1.0)[3] == 0.0
    assert _mu(orc, w, 2 * MEC2)[3] == 0.0
    vals = [_mu(orc, w, E)[3] for E in np.linspace(1.05, 20, 50)]
    assert all(v > 0 for v in vals) and all(np.diff(vals) > 0)
    assert 1e-3 < _mu(orc, w, 5.0)[3] < 1e-2        # textbook magnitude, a few 1e-3 cm^2/g
    # Z^2 per atom
    cu = {"Z": [29], "A": [63.546], "w": [1.0], "I_eV": 1}
    o = {"Z": [8], "A": [15.999], "w": [1.0], "I_eV": 1}
    assert _mu(orc, cu, 4.0)[3] / _mu(orc, o, 4.0)[3] == pytest.approx((29 / 8) ** 2 * 15.999 / 63.546, rel=1e-12)


def test_water_total_attenuation_magnitude(orc):
    """Compton-dominated water attenuation at 1 and 2 MeV matches textbook magnitudes
    (0.0707 and 0.0494 cm^2/g) within 1%."""
    assert _mu(orc, synth.WATER, 1.0)[0] == pytest.approx(0.0707, rel=0.01)
    assert _mu(orc, synth.WATER, 2.0)[0] == pytest.approx(0.0494, rel=0.01)


# ---------------------------------------------------------------- electrons
def bethe_unrestricted_textbook(m, T):
    """Unrestricted electron collision stopping power in the textbook form
    ln[tau^2 (tau+2) / (2 (I/mc^2)^2)] + F(tau), F = 1 - b^2 + [tau^2/8 - (2tau+1) ln 2]/(tau+1)^2."""
    ne = NA * sum(w * z / a for z, a, w in zip(m["Z"], m["A"], m["w"]))
    tau = T / MEC2
    b2 = 1 - 1 / (tau + 1) ** 2
    Ir = m["I_eV"] * 1e-6 / MEC2
    F = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (tau + 1) ** 2
    return 2 * math.pi * RE * RE * MEC2 * ne / b2 * (math.log(tau * tau * (tau + 2) / (2 * Ir * Ir)) + F)


def moller_dsdw(T, W):
    """Moller cross section per electron differential in the energy transfer W (cm^2/MeV)."""
    g = T / MEC2 + 1
    b2 = 1 - 1 / g ** 2
    Tp = T - W
    return 2 * math.pi * RE * RE * MEC2 / b2 * (1 / W ** 2 + 1 / Tp ** 2 + 1 / T ** 2 * ((g - 1) / g) ** 2
                                                - (2 * g - 1) / g ** 2 / (W * Tp))


@pytest.mark.parametrize("T", [0.1, 0.5, 1.0, 3.0, 6.0])
def test_bethe_two_forms_agree(orc, T):
    for m in (synth.WATER, synth.COPPER, synth.GOS):
        assert orc.lib().orc_lcol(ct.byref(_mat(orc, m)), T, 0, 0.2) == pytest.approx(
            bethe_unrestricted_textbook(m, T), rel=1e-12)


def test_stopping_power_textbook_magnitude(orc):
    """Water collision stopping power (ESTAR-like magnitudes; no density effect here,
    which matters by ~1% at 1 MeV): 4.115 at 0.1 MeV, 1.849 at 1 MeV (MeV cm^2/g)."""
    w = _mat(orc, synth.WATER)
    assert orc.lib().orc_lcol(ct.byref(w), 0.1, 0, 0.2) == pytest.approx(4.115, rel=0.015)
    assert orc.lib().orc_lcol(ct.byref(w), 1.0, 0, 0.2) == pytest.approx(1.849, rel=0.02)


@pytest.mark.parametrize("T", [0.45, 1.0, 2.5, 6.0])
def test_restricted_plus_hard_moller_moment_is_unrestricted(orc, T):
    """L_unrestricted - L_restricted(Wc) = n_e int_{Wc}^{T/2} W dsigma/dW dW, and
    Sigma_Moller = n_e int_{Wc}^{T/2} dsigma/dW dW (30-digit quadratures of the
    differential in W)."""
    import mpmath as mp
    mp.mp.dps = 30
    m = synth.WATER
    ne = mp.mpf(NA) * sum(mp.mpf(w) * z / mp.mpf(a) for z, a, w in zip(m["Z"], m["A"], m["w"]))
    Tm = mp.mpf(T)
    g = Tm / mp.mpf(MEC2) + 1
    b2 = 1 - 1 / g ** 2

    def d(W):
        Tp = Tm - W
        return 2 * mp.pi * mp.mpf(RE) ** 2 * mp.mpf(MEC2) / b2 * (
            1 / W ** 2 + 1 / Tp ** 2 + ((g - 1) / g) ** 2 / Tm ** 2 - (2 * g - 1) / g ** 2 / (W * Tp))

    pts = [mp.mpf("0.2"), (mp.mpf("0.2") + Tm / 2) / 2, Tm / 2]
    L = orc.lib()
    mm = _mat(orc, m)
    diff = L.orc_lcol(ct.byref(mm), T, 0, 0.2) - L.orc_lcol(ct.byref(mm), T, 1, 0.2)
    assert diff == pytest.approx(float(ne * mp.quad(lambda W: W * d(W), pts)), rel=1e-11)
    assert L.orc_sigma_moller(ct.byref(mm), T, 0.2) == pytest.approx(float(ne * mp.quad(d, pts)), rel=1e-11)


def test_moller_below_threshold(orc):
    mm = _mat(orc, synth.WATER)
    assert orc.lib().orc_sigma_moller(ct.byref(mm), 0.4, 0.2) == 0.0
    assert orc.lib().orc_sigma_moller(ct.byref(mm), 0.41, 0.2) > 0.0


@pytest.mark.parametrize("T", [0.6, 2.0, 5.0])
def test_moller_sampler_chi2(orc, T):
    rng = np.random.default_rng(int(T * 100))
    n = 50_000
    L = orc.lib()
    W = np.array([L.orc_moller_sample(T, 0.2, x) for x in rng.random(n)])
    assert W.min() >= 0.2 and W.max() <= T / 2
    edges = np.linspace(0.2, T / 2, 31)
    obs, _ = np.histogram(W, edges)
    tot = integrate.quad(lambda w: moller_dsdw(T, w), 0.2, T / 2, epsrel=1e-12)[0]
    exp = np.array([integrate.quad(lambda w: moller_dsdw(T, w), a, b, epsrel=1e-12)[0]
                    for a, b in zip(edges[:-1], edges[1:])]) / tot * n
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3


def test_brems_total_is_integral_of_1_over_k(orc):
    """Sigma_brems = int_{kc}^{T} S_rad/(T k) dk, and S_rad = (sigma * T / ln(T/kc)) is
    proportional to the unrestricted collision power times Z_eff T / 800."""
    m = synth.GOS
    mm = _mat(orc, m)
    L = orc.lib()
    zeff = sum(w * z * z / a for z, a, w in zip(m["Z"], m["A"], m["w"])) / \
        sum(w * z / a for z, a, w in zip(m["Z"], m["A"], m["w"]))
    for T in (0.3, 1.0, 4.0):
        srad = bethe_unrestricted_textbook(m, T) * zeff * T / 800.0
        assert L.orc_sigma_brems(ct.byref(mm), T, 0.01) == pytest.approx(srad / T * math.log(T / 0.01), rel=1e-10)
        # soft radiative part of the restricted loss is S_rad * kc / T
        soft = L.orc_lres(ct.byref(mm), T, 0.2, 0.01) - L.orc_lcol(ct.byref(mm), T, 1, 0.2)
        assert soft == pytest.approx(srad * 0.01 / T, rel=1e-9)


def test_range_quadrature_and_inverse(orc):
    L = orc.lib()
    for m in (synth.WATER, synth.COPPER, synth.GOS):
        mm = _mat(orc, m)
        for lo, hi in ((0.2, 1.0), (0.18, 0.2), (0.36, 0.44), (1.0, 6.0)):
            ref = integrate.quad(lambda t: 1.0 / L.orc_lres(ct.byref(mm), t, 0.2, 0.01), lo, hi,
                                 points=[0.4] if lo < 0.4 < hi else None, epsrel=1e-12, limit=200)[0]
            assert L.orc_range_diff(ct.byref(mm), lo, hi, 0.2, 0.01) == pytest.approx(ref, rel=1e-9)
        for T0, T1 in ((1.0, 0.9), (0.45, 0.38), (6.0, 5.5), (0.25, 0.21)):
            dR = L.orc_range_diff(ct.byref(mm), T1, T0, 0.2, 0.01)
            assert L.orc_range_inverse(ct.byref(mm), T0, dR, 0.2, 0.01) == pytest.approx(T1, rel=1e-10)


def test_csda_range_textbook_magnitude(orc):
    """Water CSDA range 0.2 -> 1 MeV: ESTAR-like 0.437 - 0.045 = 0.39 g/cm^2 (within 5%)."""
    mm = _mat(orc, synth.WATER)
    assert orc.lib().orc_range_diff(ct.byref(mm), 0.2, 1.0, 0.2, 0.01) == pytest.approx(0.392, rel=0.05)


def test_radiation_length(orc):
    """Dahl's X0 for water is within 1% of the tabulated 36.08 g/cm^2."""
    assert orc.lib().orc_x0(ct.byref(_mat(orc, synth.WATER))) == pytest.approx(36.08, rel=0.01)


def test_highland_scaling(orc):
    L = orc.lib()
    a = L.orc_highland(1.0, 0.1, 36.0)
    # zero thickness scatters nothing; thicker steps scatter more; faster electrons less
    assert L.orc_highland(1.0, 0.0, 36.0) == 0.0
    assert L.orc_highland(1.0, 0.4, 36.0) > a > L.orc_highland(3.0, 0.1, 36.0)
    # a 1 MeV electron through 0.1 g/cm^2 of water (a quarter of its range) is
    # deflected by tens of degrees
    assert 0.3 < a < 0.55
    # theta0 scales roughly as sqrt(thickness): 4x thicker gives ~2x wider
    assert 1.8 < L.orc_highland(1.0, 0.4, 36.0) / a < 2.4


# ---------------------------------------------------------------- HU mapping
def test_hu_mapping_reading(orc):
    hu = np.array([-1024, -1000, -951, -950, -700, -201, -200, 0, 299, 300, 1000, 3000], dtype=np.int16)
    m, rho = orc.map_hu(hu, synth.HU_CURVE, synth.HU_RANGES)
    assert list(m) == [0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3]
    np.testing.assert_allclose(rho, [0.0, 0.0, 0.049, 0.05, 0.3, 0.799, 0.8, 1.0, 1.1794, 1.18, 1.6, 2.8],
                               rtol=1e-12, atol=1e-15)
