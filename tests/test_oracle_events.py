"""Pins of the oracle read from its event trace and its physics entry points (CPU only):
interaction kinematics against energy and momentum conservation, the pair split and the
annihilation photons against uniform and isotropic laws, the bremsstrahlung sampler against
the 1/k law and the radiative energy balance, the Highland width at its closed-form special
cases, the multiple-scattering angle against the Rayleigh law, the hinge point, the hard-event
rate against the integral of the cross section along the tracks, brute-force re-binning of
the deposits on a tiny grid, and the effect of the step floor.  The checks themselves live in
tests/_oracle_pins.py so that the mutation test runs them on planted mistakes too."""
import pytest

from tests import _oracle_pins as pins


def test_compton_kinematics(orc):
    pins.pin_compton_kinematics(orc)


def test_pair_and_annihilation(orc):
    pins.pin_pair_and_annihilation(orc)


def test_moller_and_brems_kinematics(orc):
    pins.pin_moller_and_brems_kinematics(orc)


def test_brems_sampler_is_one_over_k(orc):
    pins.pin_brems_sampler(orc)


def test_brems_energy_balance(orc):
    pins.pin_brems_energy_balance(orc)


def test_radiative_stopping_power_magnitude(orc):
    pins.pin_srad_magnitude(orc)


def test_highland_special_cases(orc):
    pins.pin_highland_special_cases(orc)


def test_msc_angle_is_rayleigh_and_hinge_uniform(orc):
    pins.pin_msc_rayleigh_and_hinge(orc)


def test_sigma_hard_majorant(orc):
    pins.pin_sigma_hard_majorant(orc)


def test_hard_event_rate_matches_cross_section_integral(orc):
    pins.pin_hard_event_rate(orc)


def test_tiny_grid_rebinning(orc):
    pins.pin_tiny_grid_rebinning(orc)


def test_step_floor_effect_within_statistics(orc):
    g, rel, sd = pins.pin_step_floor_bias(orc)
    print(f"step floor 0.05 vs 0: z-gate {g}; scoring-layer total differs by {rel:+.4%} +- {sd:.4%}")


def test_goldens_come_from_the_current_oracle():
    """The stored oracle images (tests/golden/*.npz) were written by the oracle source as it
    stands: a change to its arithmetic must be followed by running make_oracle_goldens.py."""
    import glob
    import os

    import numpy as np

    from tests.golden.make_oracle_goldens import GOLDENS, oracle_source_sha
    here = os.path.join(os.path.dirname(__file__), "golden")
    files = sorted(glob.glob(os.path.join(here, "oracle_*.npz")))
    assert sorted(os.path.basename(f)[:-4] for f in files) == sorted(GOLDENS)
    for f in files:
        d = np.load(f)
        assert str(d["oracle_sha"]) == oracle_source_sha(), f
        g = GOLDENS[os.path.basename(f)[:-4]]
        assert int(d["histories"]) == g["histories"] and int(d["seed"]) == g["seed"]
