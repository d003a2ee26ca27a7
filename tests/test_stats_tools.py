"""Pins of the comparison tools on images with known answers."""
import numpy as np

from tests._stats import gamma_pass, rebin, sigma_bar, z_gate


def test_gamma_identical_and_scaled():
    y, x = np.mgrid[0:64, 0:64]
    ref = np.exp(-((x - 32.0) ** 2 + (y - 30.0) ** 2) / 200.0)
    assert gamma_pass(ref, ref, 0.1) == 1.0
    assert gamma_pass(ref, ref * 1.019, 0.1, dta=1e-6) == 1.0      # within 2% of max everywhere
    assert gamma_pass(ref, ref * 1.05, 0.1, dta=1e-6) < 1.0         # 5% off near the peak fails


def test_gamma_shift_against_distance_criterion():
    """A steep edge shifted by 1.5 mm passes 2%/2 mm but fails 2%/1 mm near the edge."""
    x = np.arange(200) * 0.05                     # 0.5 mm pixels
    ref = np.tile((x > 5.0).astype(float) * 0.9 + 0.1, (20, 1))
    evl = np.tile((x > 5.15).astype(float) * 0.9 + 0.1, (20, 1))
    assert gamma_pass(ref, evl, 0.05, dd=0.02, dta=0.2) == 1.0
    assert gamma_pass(ref, evl, 0.05, dd=0.02, dta=0.1) < 1.0


def test_zgate_on_gaussian_noise():
    rng = np.random.default_rng(1)
    d = np.full((64, 64), 10.0)
    v = np.full((64, 64), 0.04)
    a = d + rng.normal(0, 0.2, d.shape)
    b = d + rng.normal(0, 0.2, d.shape)
    assert z_gate(a, v, b, v)["ok"]
    assert not z_gate(a * 1.02, v, b, v)["ok"]                    # a 2% bias is 7 sigma per pixel
    assert not z_gate(a, v * 4, b, v * 4)["ok"]                    # overstated variance: sd(z) << 1


def test_rebin_and_sigma_bar():
    a = np.arange(16.0).reshape(4, 4)
    assert rebin(a, 2).tolist() == [[10.0, 18.0], [42.0, 50.0]]
    m = np.array([[1.0, 0.05], [0.8, 0.6]])
    v = np.array([[1e-4, 1.0], [6.4e-5, 3.6e-5]])
    assert abs(sigma_bar(m, v, 0.5) - np.mean([0.01, 0.01, 0.01])) < 1e-12
