"""The seeded workload generators produce the stated shapes and values."""
import numpy as np

from paper_2510_24154_amd import synth


def test_kerma_water_shapes():
    c = synth.kerma_water()
    assert c["phantom"]["shape"] == (100, 100, 100) and c["phantom"]["rho"].size == 10 ** 6
    assert (c["epid"]["npx_u"], c["epid"]["npx_v"], c["epid"]["pitch_u"]) == (128, 128, 0.2)
    assert [l["t"] for l in c["epid"]["layers"]] == [0.2, 0.03, 0.1]
    assert c["epid"]["front_z"] == 70.0


def test_coupled_hetero_geometry():
    c = synth.coupled_hetero()
    P = c["phantom"]
    assert P["shape"] == (256, 256, 128) and P["hu"].size == 256 * 256 * 128
    assert set(np.unique(P["hu"])) <= {0, -700, 1000} and (P["hu"] == -700).any() and (P["hu"] == 1000).any()
    assert abs(P["origin"][2] + 0.5 * 128 * 0.2 - 100.0) < 1e-9          # centred on the isocentre
    E = c["epid"]
    assert (E["npx_u"], E["npx_v"]) == (768, 1024) and abs(E["pitch_u"] - 0.039) < 1e-12
    z = E["front_z"] + sum(l["t"] for l in E["layers"][:2]) + 0.5 * E["layers"][2]["t"]
    assert abs(z - 150.0) < 1e-9                                          # phosphor mid-plane at SID
    edges, w = c["source"]["edges"], c["source"]["weights"]
    assert len(w) == 118 and abs(edges[0] - 0.1) < 1e-12 and abs(edges[-1] - 6.0) < 1e-9
    assert abs(w.sum() - 1.0) < 1e-12 and (w > 0).all()


def test_seeded_and_reproducible():
    a, b = synth.ellipsoid_list(2), synth.ellipsoid_list(2)
    assert a == b and a != synth.ellipsoid_list(3)


def test_mlc_segments_counts():
    ap = synth.mlc_segments()
    n = ap["counts"].astype(np.int64)
    assert n.sum() == 300_000_000 and n.min() >= 1_000_000 and n.max() <= 50_000_000
    assert ap["a"].shape == (40, 60) and (ap["b"] >= ap["a"]).all()
    assert np.all(ap["b"] - ap["a"] <= 10.0)


def test_mixed_denoiser_fields():
    """Even seeds keep the single-segment ellipsoid field; odd seeds of the mixed recipe give
    a thorax-like phantom of the large case's extents under 5-20 segments."""
    from paper_2510_24154_amd import synth
    even = synth.denoise_field(4, mixed=True)
    assert even["source"]["aperture"]["a"].shape[0] == 1
    odd = synth.denoise_field(5, mixed=True)
    ph = odd["phantom"]
    assert ph["shape"] == (128, 128, 50) and ph["spacing"] == (0.4, 0.4, 0.4)
    assert set(np.unique(ph["hu"])) <= {-1000, -750, 40, 60, 800}
    assert (ph["hu"] == -750).sum() > 0 and (ph["hu"] == 800).sum() > 0
    ap = odd["source"]["aperture"]
    n_seg = ap["a"].shape[0]
    assert 5 <= n_seg <= 20 and int(ap["counts"].sum()) == 1_000_000 * n_seg
    # the same seed gives the same field
    again = synth.denoise_field(5, mixed=True)
    assert np.array_equal(again["phantom"]["hu"], ph["hu"]) and np.array_equal(again["source"]["aperture"]["a"], ap["a"])
