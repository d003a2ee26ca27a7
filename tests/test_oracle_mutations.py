"""Mutation check of the oracle's pins (CPU only): each case plants one plausible mistake in
a copy of the oracle's source, builds it to a temporary library, and runs the pin that must
catch it against that build.  A pin that still passed would be no pin for that part."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import _oracle_pins as pins
from tests import test_oracle_physics as phys
from tests import test_oracle_transport as trans

SRC = os.path.join(os.path.dirname(oracle.__file__), "epid_oracle.c")

# (name, [(text in epid_oracle.c, replacement)], pin that must fail)
MUTANTS = [
    ("Compton angle for the sampled E'",
     [("double ct = 1.0 - (1.0 / eps - 1.0) / k;", "double ct = 1.0 - (1.0 / eps - 1.0) / (2.0 * k);")],
     pins.pin_compton_kinematics),
    ("Compton electron energy",
     [("double Ep = eps * E, T = E - Ep;", "double Ep = eps * E, T = E - 0.5 * Ep;")],
     pins.pin_compton_kinematics),
    ("Klein-Nishina CDF term",
     [("+ c * log(e / e0) + a * a * (1.0 / e0 - 1.0 / e);", "+ c * log(e / e0) + a * (1.0 / e0 - 1.0 / e);")],
     lambda orc: phys.test_kn_sampler_chi2(orc, 2.0)),
    ("delta-ray polar angle",
     [("double cd = sqrt(W * (T + 2.0 * MEC2) / (T * (W + 2.0 * MEC2)));",
       "double cd = sqrt(W * (T + MEC2) / (T * (W + 2.0 * MEC2)));")],
     pins.pin_moller_and_brems_kinematics),
    ("Moller azimuths not opposite",
     [("rotate(e.d, fmin(cp, 1.0), sqrt(fmax(0.0, 1.0 - cp * cp)), phi + PI);",
       "rotate(e.d, fmin(cp, 1.0), sqrt(fmax(0.0, 1.0 - cp * cp)), phi);")],
     pins.pin_moller_and_brems_kinematics),
    ("pair energy split not uniform",
     [("double tm = orng_u(&c->rng) * T, tp = T - tm;", "double tm = sqrt(orng_u(&c->rng)) * T, tp = T - tm;")],
     pins.pin_pair_and_annihilation),
    ("annihilation photons not isotropic",
     [("double ct = 2.0 * orng_u(rng) - 1.0, phi = 2.0 * PI * orng_u(rng);",
       "double ct = orng_u(rng), phi = 2.0 * PI * orng_u(rng);")],
     pins.pin_pair_and_annihilation),
    ("bremsstrahlung sampler exponent",
     [("return kcut * exp(xi * log(T / kcut));", "return kcut * exp(xi * xi * log(T / kcut));")],
     pins.pin_brems_sampler),
    ("radiative stopping power without Z_eff",
     [("return orc_lcol(m, T, 0, 0.0) * mat_zeff(m) * T / BREM_K;", "return orc_lcol(m, T, 0, 0.0) * T / BREM_K;")],
     pins.pin_srad_magnitude),
    ("Highland log term without beta^2",
     [("double br = 1.0 + 0.038 * log(x / (X0 * b2));", "double br = 1.0 + 0.038 * log(x / X0);")],
     pins.pin_highland_special_cases),
    ("Highland constant",
     [("return 13.6 / bcp * sqrt(x / X0) * br;", "return 14.1 / bcp * sqrt(x / X0) * br;")],
     pins.pin_highland_special_cases),
    ("scattering angle not Rayleigh(theta0)",
     [("* sqrt(-2.0 * log(xi3));", "* sqrt(-log(xi3));")],
     pins.pin_msc_rayleigh_and_hinge),
    ("hinge at the step's midpoint",
     [("h[a] = e.p[a] + xi2 * s * e.d[a];", "h[a] = e.p[a] + 0.5 * s * e.d[a];")],
     pins.pin_msc_rayleigh_and_hinge),
    ("hard-event distance without the density",
     [("double s_hard = smax > 0 ? -log(xi1) / (rho * smax) : INFINITY;",
       "double s_hard = smax > 0 ? -log(xi1) / smax : INFINITY;")],
     pins.pin_hard_event_rate),
    ("Moller events turned into bremsstrahlung",
     [("if (u < sm) {\n                    c->cnt->n_moller++;", "if (u < 0.5 * sm) {\n                    c->cnt->n_moller++;")],
     pins.pin_hard_event_rate),
    ("hard-event majorant from the start energy only",
     [("return a > b ? a : b;", "return a;")],
     pins.pin_sigma_hard_majorant),
    ("pixel index transposed",
     [("int pix = (int)fv * cf->npx_u + (int)fu;", "int pix = (int)fu * cf->npx_v + (int)fv;")],
     pins.pin_tiny_grid_rebinning),
    ("voxel axes swapped in photon tracking",
     [("long v = ((long)idx[2] * cf->ny + idx[1]) * cf->nx + idx[0];\n                int m = cf->vox_mat[v];",
       "long v = ((long)idx[2] * cf->ny + idx[0]) * cf->nx + idx[1];\n                int m = cf->vox_mat[v];")],
     trans.test_pixel_resolved_absorption_parallel),
]


@pytest.fixture(scope="module")
def workdir():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp(prefix="orc_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def build_mutant(workdir, i, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, f"mutation site not found exactly once: {old!r}"
        src = src.replace(old, new)
    c, so = os.path.join(workdir, f"m{i}.c"), os.path.join(workdir, f"m{i}.so")
    open(c, "w").write(src)
    shutil.copy(os.path.join(os.path.dirname(SRC), "epid_oracle.h"), workdir)
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-o", so, c, "-lm", "-lpthread"])
    return so


@pytest.mark.parametrize("i", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_its_pin(workdir, i):
    name, edits, pin = MUTANTS[i]
    so = build_mutant(workdir, i, edits)
    with oracle.using(so):
        with pytest.raises(AssertionError):
            pin(oracle)
