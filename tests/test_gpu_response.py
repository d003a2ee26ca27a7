"""GPU parity of the dose-response correction (Sec. 2.2, Sec. 3.1) through the C ABI: the
device radiological-thickness map against the oracle's FP64 Siddon trace (every pixel, from
test-sized grids up to the full 256x256x128 phantom with its 1024x768 image), the field size,
and k(t, s) * image against the oracle's bilinear Table 1.

The engine receives geometry as FP32 through the ABI, so the oracle gets the same values
rounded to FP32; the remaining differences are the packed voxel densities (within 2^-21
relative) and FP64 summation order, hence the 1e-6 relative tolerance."""
import copy

import numpy as np
import pytest

from paper_2510_24154_amd import synth
from tests.test_oracle_response import aperture, golden_table1, slab_case

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_24154_amd as E
    return E


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def as_engine_sees_it(cfg):
    """The workload with every geometric input rounded to FP32, as the ABI receives it."""
    c = copy.deepcopy(cfg)
    P = c["phantom"]
    P["spacing"] = tuple(f32(P["spacing"]))
    P["origin"] = tuple(f32(P["origin"]))
    if P["kind"] == "direct":
        P["rho"] = f32(P["rho"])
    Ep = c["epid"]
    for key in ("front_z", "pitch_u", "pitch_v"):
        Ep[key] = float(f32(Ep[key]))
    for L in Ep["layers"]:
        L["t"], L["rho"] = float(f32(L["t"])), float(f32(L["rho"]))
    b = c["source"]["beam"]
    b["src"] = tuple(f32(b["src"]))
    b["iso_z"] = float(f32(b["iso_z"]))
    return c


def engine_for(E, cfg):
    eng = E.Engine(0, seed=1).configure(cfg, batches=16, max_chunk=1 << 16)
    eng.bind()
    return eng


def heterogeneous_grid():
    rng = np.random.default_rng(11)
    cfg = synth.kerma_water(npx=24, pitch=1.0)
    cfg["phantom"] = {"kind": "direct", "shape": (5, 4, 3), "spacing": (3.0, 4.5, 6.0), "origin": (-6.0, -8.0, 70.0),
                      "mat": np.zeros(60, np.uint8), "rho": rng.uniform(0.0, 2.0, 60)}
    cfg["epid"]["front_z"] = 140.0
    cfg["source"]["beam"] = {"kind": 1, "src": (3.0, -2.0, 0.0), "iso_z": 100.0}
    return cfg


CASES = {
    "parallel_water_box": lambda: synth.kerma_water(npx=32, pitch=0.8),
    "oblique_slabs": lambda: slab_case([(1.0, 1.0)] * 5 + [(0.3, 1.0)] * 7 + [(1.85, 1.0)] * 3 + [(0.0012, 1.0)] * 2),
    "rays_beside_the_box": lambda: slab_case([(1.0, 1.0)] * 4, xy=4.0, npx=40, pitch=2.0),
    "random_unequal_grid": heterogeneous_grid,
    "hu_phantom_small": synth.coupled_hetero_small,
}


@pytest.mark.parametrize("name", list(CASES))
def test_radiological_thickness_matches_oracle(E, orc, name):
    cfg = CASES[name]()
    print(f"[radthick] {name}", flush=True)
    eng = engine_for(E, cfg)
    dev = eng.radiological_thickness().cpu().numpy()
    ref = orc.radiological_thickness(as_engine_sees_it(cfg))
    assert dev.shape == ref.shape
    err = np.abs(dev - ref) - (TOL * ref + 1e-9)
    assert np.all(err <= 0), (name, float(np.max(np.abs(dev - ref))), np.unravel_index(np.argmax(err), err.shape))
    assert np.count_nonzero(ref) > 0


def test_radiological_thickness_full_size(E, orc):
    """The benchmark's phantom and image: 256x256x128 voxels of 2 mm, 1024x768 pixels of
    0.39 mm, every one of the 786 432 rays against the oracle."""
    cfg = synth.coupled_hetero()
    eng = E.Engine(0, seed=1).configure(cfg, batches=16, max_chunk=1 << 20)
    eng.bind()
    dev = eng.radiological_thickness().cpu().numpy()
    ref = orc.radiological_thickness(as_engine_sees_it(cfg))
    rel = np.abs(dev - ref) / np.maximum(ref, 1e-9)
    print("full-size radiological thickness: max rel diff", rel.max(), "range", ref.min(), ref.max())
    assert np.all(np.abs(dev - ref) <= TOL * ref + 1e-9)


@pytest.mark.parametrize("segments", [
    [[(20, 39, -5.0, 5.0)]],
    [[(10, 49, -5.0, 5.0)]],
    [[(20, 23, -7.0, -3.0)], [(40, 43, 1.0, 9.0)]],
])
def test_field_size_matches_oracle(E, orc, segments):
    cfg = synth.kerma_water(npx=16, pitch=1.0)
    cfg["source"]["aperture"] = aperture(segments)
    eng = engine_for(E, cfg)
    assert abs(eng.field_size() - orc.equivalent_square(as_engine_sees_it(cfg))) < 1e-6


@pytest.mark.parametrize("s", [2.0, 5.0, 7.5, 10.0, 13.3, 20.0, 24.0])
def test_dose_response_matches_oracle_table1(E, orc, s):
    """k(t, s) * image for thicknesses spanning and exceeding Table 1, at field sizes at,
    between and outside its nodes."""
    import torch
    cfg = synth.kerma_water(npx=64, pitch=0.5)
    eng = engine_for(E, cfg)
    t_nodes, s_nodes, k = synth.response_table_1()
    rng = np.random.default_rng(int(s * 10))
    th = rng.uniform(-3.0, 30.0, (64, 64))
    th[0, :5] = t_nodes                                   # the nodes themselves
    img = rng.uniform(0.0, 2.0, (64, 64))
    out = eng.dose_response(torch.as_tensor(img), torch.as_tensor(th), s, t_nodes, s_nodes, k).cpu().numpy()
    ref = img * orc.response_factor(t_nodes, s_nodes, k, th, s)
    assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref)) + 1e-300
    if s in s_nodes:   # at a node of both axes the factor is the printed value
        j = list(s_nodes).index(s)
        tj, sj, kj = golden_table1()
        assert np.allclose(out[0, :5] / img[0, :5], kj[j], rtol=1e-15, atol=0)


def test_dose_response_rejects_bad_tables(E):
    import torch
    cfg = synth.kerma_water(npx=8, pitch=1.0)
    eng = engine_for(E, cfg)
    z = torch.zeros(8, 8, dtype=torch.float64)
    t_nodes, s_nodes, k = synth.response_table_1()
    with pytest.raises(E.EpidmcError):
        eng.dose_response(z, z, 10.0, t_nodes[::-1], s_nodes, k)   # descending nodes
    with pytest.raises(E.EpidmcError):
        eng.dose_response(z, z, 10.0, np.arange(65.0), s_nodes, np.ones((4, 65)))   # over 64 nodes
    with pytest.raises(E.EpidmcError):
        eng.dose_response(z, z, float("nan"), t_nodes, s_nodes, k)


def test_radiological_thickness_large_phantom(E, orc):
    """The large case: 512x512x200 voxels of 1 mm (52 M voxels, 210 MB packed, larger than one
    XCD's L2 many times over), every pixel of the 1024x768 image against the oracle."""
    cfg = synth.large_anthropomorphic(total=1_000_000)
    eng = E.Engine(0, seed=1).configure(cfg, batches=16, max_chunk=1 << 20)
    eng.bind()
    dev = eng.radiological_thickness().cpu().numpy()
    ref = orc.radiological_thickness(as_engine_sees_it(cfg))
    print("large phantom radiological thickness range", ref.min(), ref.max())
    assert ref.max() > 15.0   # rays cross the body
    assert np.all(np.abs(dev - ref) <= TOL * ref + 1e-9)
    # the field size of the 60-segment union matches as well
    assert abs(eng.field_size() - orc.equivalent_square(as_engine_sees_it(cfg))) < 1e-6


def test_large_case_transport_energy_ledger(E):
    """Coupled transport through the large phantom under the 60-segment field (scaled to 2e5
    histories): every history's ledger closes to 1e-9 on the device."""
    cfg = synth.large_anthropomorphic(total=200_000)
    eng = E.Engine(0, seed=3).configure(cfg, batches=16, max_chunk=1 << 17, diag=True)
    eng.bind()
    eng.run(200_000)
    c = eng.counters()
    print("large case: ledger", c["max_ledger_resid"], "woodcock steps/history", c["woodcock_steps"] / 2e5)
    assert c["max_ledger_resid"] < 1e-9
    m, v = eng.image()
    assert bool(np.isfinite(m.cpu().numpy()).all()) and float(m.sum()) > 0


def test_dose_response_64x64_lut_matches_oracle(E, orc):
    """The large case's correction table: Table 1 resampled by the engine onto 64 thickness
    nodes over 0-40 cm and 64 field-size nodes over 2-25 cm (both containing Table 1's nodes),
    applied on the device bilinear and clamped, against the oracle evaluating Table 1 itself:
    the same function, so the same corrected image."""
    import torch
    t, s, k = golden_table1()
    t_nodes, s_nodes = synth.lut64_nodes()
    lut = E.resample_response_table(t, s, k, t_nodes, s_nodes)
    rng = np.random.default_rng(64)
    cfg = synth.kerma_water(npx=64, pitch=0.5)
    eng = engine_for(E, cfg)
    th = rng.uniform(-5.0, 45.0, (64, 64))
    img = rng.uniform(0.0, 2.0, (64, 64))
    for sv in (1.0, 2.0, 5.0, 9.37, 20.0, 25.0, 30.0):
        out = eng.dose_response(torch.as_tensor(img), torch.as_tensor(th), sv, t_nodes, s_nodes, lut).cpu().numpy()
        ref = img * orc.response_factor(t, s, k, th, sv)
        assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref)), sv
