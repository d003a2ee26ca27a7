"""GPU parity tests through the C ABI: the HIP transport against the CPU oracle on
the same seeded workloads (different random streams), and against closed forms.

Parity is statistical (Monte Carlo): per-pixel standard scores of the difference,
judged as a population (z-gate), plus exact closed forms where they exist, the
per-history energy ledger, and bit-exact invariants of the fixed-point tally."""
import copy
import math
import os

import numpy as np
import pytest

from paper_2510_24154_amd import synth
from tests._stats import gamma_pass, rebin, sigma_bar, z_gate

pytestmark = pytest.mark.gpu
THREADS = max(1, min(16, os.cpu_count() or 1))
_ORACLE_CACHE = {}


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_24154_amd as E
    return E


def oracle_image(orc, key, cfg, n, seed=1001):
    if key not in _ORACLE_CACHE:
        print(f"[oracle] {key}: {n} histories on {THREADS} threads", flush=True)
        _ORACLE_CACHE[key] = orc.run(cfg, n, seed=seed, threads=THREADS)
    return _ORACLE_CACHE[key]


def gpu_image(E, cfg, n, seed=1, **kw):
    kw.setdefault("batches", 64)
    kw.setdefault("max_chunk", 1 << 22)
    eng = E.Engine(0, seed=seed).configure(cfg, **kw)
    eng.bind()
    eng.run(n)
    m, v = eng.image()
    return m.cpu().numpy(), v.cpu().numpy(), eng


def mu(orc, m, En, mask):
    import ctypes as ct
    out = np.zeros(4)
    orc.lib().orc_photon_mu(ct.byref(orc.material(m)), En, out.ctypes.data)
    return sum(out[1 + i] for i in range(3) if mask >> i & 1)


def test_transmission_water_box(E, orc):
    """Woodcock tracking in the phantom: unscattered primaries behind 20 cm of water
    are exp(-20 mu) (binomial z)."""
    n = 4_000_000
    _, _, eng = gpu_image(E, synth.kerma_water(), n)
    c = eng.counters()
    p = math.exp(-20.0 * mu(orc, synth.WATER, 2.0, 0b011))
    z = (c["unscattered_at_epid"] - n * p) / math.sqrt(n * p * (1 - p))
    assert abs(z) < 4, z


def test_transmission_heterogeneous_slabs(E, orc):
    """Delta tracking through bone, lung, air and water slabs against exp(-sum mu rho t):
    exercises the majorant across materials and densities."""
    cfg = synth.coupled_hetero_small()
    cfg["physics"]["coupled"] = 0
    cfg["source"] = synth.kerma_water()["source"]
    cfg["source"]["edges"] = np.array([0.6, 0.6])
    slabs = [(2, 1.0, 10), (3, 1.6, 7), (1, 0.3, 20), (3, 1.85, 3), (0, 0.0012, 5), (2, 1.0, 15)]
    nz = sum(s[2] for s in slabs)
    mats = np.concatenate([np.full(s[2], s[0], np.uint8) for s in slabs])
    rhos = np.concatenate([np.full(s[2], s[1], np.float32) for s in slabs])
    cfg["phantom"] = {"kind": "direct", "shape": (4, 4, nz), "spacing": (5.0, 5.0, 0.2), "origin": (-10.0, -10.0, 0.0),
                      "mat": np.repeat(mats, 16), "rho": np.repeat(rhos, 16)}
    n = 4_000_000
    _, _, eng = gpu_image(E, cfg, n)
    c = eng.counters()
    tau = sum(mu(orc, cfg["materials"][m], 0.6, 0b011) * float(np.float32(rho)) * k * 0.2 for m, rho, k in slabs)
    p = math.exp(-tau)
    z = (c["unscattered_at_epid"] - n * p) / math.sqrt(n * p * (1 - p))
    assert abs(z) < 4, z


def pixel_resolved_case(orc):
    """Photoelectric-only 30 keV parallel beam through a 4x4 set of density columns onto a
    lone 30 um phosphor; returns the workload and each pixel's exact mean deposit."""
    En = 0.03
    cfg = synth.kerma_water()
    cfg["physics"] = {"coupled": 0, "proc_mask": 0b010, "pcut": 0.01, "ecut": 0.2}
    cfg["source"]["edges"] = np.array([En, En])
    col = np.random.default_rng(7).uniform(0.1, 1.0, (4, 4))
    cfg["phantom"] = {"kind": "direct", "shape": (4, 4, 4), "spacing": (2.5, 2.5, 1.0), "origin": (-5.0, -5.0, 0.0),
                      "mat": np.zeros(64, np.uint8), "rho": np.tile(col.reshape(-1), 4).astype(np.float32)}
    cfg["epid"] = {"layers": [{"mat": 2, "t": 0.003, "rho": 7.44}], "scoring": 0, "front_z": 20.0,
                   "npx_u": 16, "npx_v": 16, "pitch_u": 0.625, "pitch_v": 0.625}
    mw, mg = mu(orc, synth.WATER, En, 2), mu(orc, synth.GOS, En, 2)
    absorb = 1 - math.exp(-mg * 7.44 * 0.003)
    rho32 = col.astype(np.float32).astype(np.float64)
    expect = np.array([[En * (0.625 ** 2 / 100.0) * math.exp(-mw * rho32[v // 4, u // 4] * 4.0) * absorb
                        for u in range(16)] for v in range(16)])
    return cfg, expect, En


def test_pixel_resolved_absorption(E, orc):
    """Each pixel's mean deposit against its closed form (per-pixel binomial z); x and y
    differ, so a transposed or mirrored index fails."""
    cfg, expect, En = pixel_resolved_case(orc)
    n = 4_000_000
    mean, var, _ = gpu_image(E, cfg, n)
    p = expect / En
    z = (mean - expect) / np.sqrt(En * En * p * (1 - p) / n)
    assert np.all(np.abs(z) < 5), np.abs(z).max()
    assert abs(z.mean()) < 3 / 16 and 0.8 < z.std() < 1.2


def test_pixel_resolved_gamma_against_exact_image(E, orc):
    """Gamma gate (2%/2 mm, 10% threshold, pass rate >= 99%) of the engine's image against
    the exact expected image.  The reference carries no noise, and at 1.6e8 histories every
    pixel holds at least 2.6e5 absorptions (relative noise <= 0.2%), so a pass rate below
    99% means a bias of the order of the criterion, not noise.  Against the oracle the same gate is
    out of reach in test time: phosphor deposits are rare, and the oracle's per-pixel noise
    at a few million histories is 5-20%; the z-gates judge that comparison instead."""
    cfg, expect, _ = pixel_resolved_case(orc)
    mean, _, _ = gpu_image(E, cfg, 160_000_000, max_chunk=1 << 25)
    rate = gamma_pass(expect, mean, 0.625, dd=0.02, dta=0.2, thr=0.10)
    print("pixel-resolved gamma 2%/2 mm pass rate", rate)
    assert rate >= 0.99, rate
    # and the gate is not vacuous: the same image with a 5% gain error fails it (most pixels
    # are above 40% of the maximum, where 5% exceeds the 2% criterion)
    assert gamma_pass(expect, mean * 1.05, 0.625, dd=0.02, dta=0.2, thr=0.10) < 0.99


def test_kerma_water_zgate(E, orc):
    """Photon-only KERMA workload: GPU image against the oracle image, per 4x4-binned pixel."""
    cfg = synth.kerma_water()
    om, ov, *_ = oracle_image(orc, "kerma_water", cfg, 8_000_000)
    gm, gv, _ = gpu_image(E, cfg, 80_000_000, max_chunk=1 << 24)
    g = z_gate(gm, gv, om, ov, thr=0.10, k=4)
    print("kerma_water z-gate", g)
    assert g["ok"], g


def test_coupled_small_zgate(E, orc):
    """Coupled transport, heterogeneous phantom, 4-layer EPID: GPU vs oracle z-gate per
    4x4-binned pixel.  Binning keeps a few hundred oracle deposits per bin: with tens of
    events the skewed per-event energy makes the oracle's own mean and variance estimates
    far from Gaussian and the z spread exceeds 1 for correct code."""
    cfg = synth.coupled_hetero_small()
    om, ov, *_ = oracle_image(orc, "coupled_small", cfg, 2_000_000)
    gm, gv, eng = gpu_image(E, cfg, 60_000_000, max_chunk=1 << 23)
    g = z_gate(gm, gv, om, ov, thr=0.10, k=4)
    print("coupled_small z-gate", g, "oracle sigma-bar(4x4)", sigma_bar(rebin(om, 4), rebin(ov, 4)))
    assert g["ok"], g


def test_coupled_energy_ledger(E):
    """Per history: incident energy = deposits + escapes + net rest energy, on the device."""
    cfg = synth.coupled_hetero_small()
    eng = E.Engine(0, seed=5).configure(cfg, batches=16, max_chunk=1 << 17, diag=True)
    eng.bind()
    eng.run(300_000)
    c = eng.counters()
    assert c["max_ledger_resid"] < 1e-9
    assert c["e_in"] > 0 and c["e_deposited"] == pytest.approx(c["e_in"], rel=1e-12)
    assert c["n_pair"] > 0 and c["n_moller"] > 0 and c["n_brems"] > 0 and c["n_annih"] > 0


def test_fixed_point_bit_reproducible_across_launch_shapes(E):
    """Fixed-point tally: the image does not depend on chunking (queue sizes, grid sizes,
    pass structure) or on repetition."""
    cfg = synth.coupled_hetero_small()
    imgs = []
    for chunk in (1 << 12, 1 << 16, 1 << 20):
        m, v, _ = gpu_image(E, cfg, 400_000, seed=11, tally=1, max_chunk=chunk)
        imgs.append((m, v))
    m2, v2, _ = gpu_image(E, cfg, 400_000, seed=11, tally=1, max_chunk=1 << 16)
    for m, v in imgs[1:] + [(m2, v2)]:
        assert np.array_equal(m, imgs[0][0]) and np.array_equal(v, imgs[0][1])
    assert imgs[0][0].sum() > 0


def test_fixed_point_same_on_a_side_stream_with_profiling(E):
    """A pass runs three particle kinds on the engine's own streams and the fourth on the
    caller's stream, which waits for the others before the next pass.  Issued on a
    non-default stream, with profiling events around every launch, a run gives the same
    fixed-point image as on the default stream, and every kind's launches are timed."""
    import torch
    cfg = synth.coupled_hetero_small()
    m0, v0, _ = gpu_image(E, cfg, 400_000, seed=11, tally=1, max_chunk=1 << 16)
    side = torch.cuda.Stream()   # default priority
    with torch.cuda.stream(side):
        eng = E.Engine(0, seed=11).configure(cfg, tally=1, batches=64, max_chunk=1 << 16)
        eng.bind()
        eng.set_profiling(True)
        eng.run(400_000)
        m, v = eng.image()
    side.synchronize()
    assert np.array_equal(m.cpu().numpy(), m0) and np.array_equal(v.cpu().numpy(), v0)
    c = eng.counters()
    assert all(n > 0 for n in c["kernel_launches"]), c["kernel_launches"]
    assert all(ms > 0 for ms in c["kernel_ms"]), c["kernel_ms"]


@pytest.mark.parametrize("n", [2, 3, 63, 65, 1025, 4097])
def test_ragged_history_counts(E, n):
    """Runs far below a wave or a chunk, and chunks with a one-history tail: the fixed-point
    image with 1024-history chunks equals the one-chunk image bit for bit, every history
    closes its energy ledger, and a run with fewer histories than variance batches (or none)
    is refused."""
    cfg = synth.coupled_hetero_small()
    m0, v0, _ = gpu_image(E, cfg, n, seed=41, tally=1, batches=2, max_chunk=1024)
    m1, v1, _ = gpu_image(E, cfg, n, seed=41, tally=1, batches=2, max_chunk=1 << 20)
    assert np.array_equal(m0, m1) and np.array_equal(v0, v1)
    assert np.isfinite(m0).all() and (m0 >= 0).all() and (v0 >= 0).all()
    eng = E.Engine(0, seed=41).configure(cfg, tally=1, batches=2, max_chunk=1024, diag=True)
    eng.bind()
    eng.run(n, first=7)
    c = eng.counters()
    assert c["error_word"] == 0 and c["max_ledger_resid"] < 1e-9
    assert c["e_in"] > 0 and c["e_deposited"] == pytest.approx(c["e_in"], rel=1e-12)
    for bad in (0, 1):
        with pytest.raises(E.EpidmcError):
            eng.run(bad)


def test_queue_overflow_is_reported_and_contained(E):
    """A phantom-electron queue shrunk to 8 particles per segment (the library's test hook)
    cannot take a pass's appends: the run stores nothing past the segments, drops what does not
    fit and returns EPIDMC_E_OVERFLOW (-7).  After a bind with the derived size the engine's
    fixed-point image equals a fresh engine's bit for bit, and its largest pass stays far
    below the derived capacity."""
    cfg = synth.coupled_hetero_small()
    n, chunk = 100_000, 1 << 16
    eng = E.Engine(0, seed=51).configure(cfg, tally=1, batches=4, max_chunk=chunk)
    eng.debug_queue_capacity(1, 8)
    eng.bind()
    with pytest.raises(E.EpidmcError) as ei:
        eng.run(n)
    assert ei.value.code == -7 and "queue overflow" in str(ei.value)
    with pytest.raises(E.EpidmcError):
        eng.debug_queue_capacity(0, 8)   # the source fills the phantom photon queue by slot
    eng.debug_queue_capacity(1, 0)
    eng.bind()
    eng.run(n)
    m1, v1 = (t.cpu().numpy() for t in eng.image())
    assert eng.counters()["queue_peak"] < 2 * chunk
    m0, v0, _ = gpu_image(E, cfg, n, seed=51, tally=1, batches=4, max_chunk=chunk)
    assert m0.sum() > 0
    assert np.array_equal(m1, m0) and np.array_equal(v1, v0)


def test_tally_modes_agree(E):
    """Same seed, same trajectories: FP64 atomics, int64 fixed point and FP32 Kahan records
    give the same image up to their rounding (fixed point 2^-32 MeV per deposit, FP32)."""
    cfg = synth.coupled_hetero_small()
    m0, v0, _ = gpu_image(E, cfg, 300_000, seed=12, tally=0)
    m1, v1, _ = gpu_image(E, cfg, 300_000, seed=12, tally=1)
    m2, v2, _ = gpu_image(E, cfg, 300_000, seed=12, tally=2)
    assert m0.sum() > 0
    np.testing.assert_allclose(m1, m0, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(m2, m0, rtol=1e-6, atol=1e-13)
    np.testing.assert_allclose(v2, v0, rtol=1e-4, atol=1e-20)


def test_segment_sum_is_field(E):
    """Histories are keyed by id: an IMRT field run in one call equals the sum of its
    segment ranges run separately (fixed point: exactly)."""
    cfg = synth.imrt_field(shape=(64, 64, 32), spacing=0.8, npx=(96, 128), pitch=0.312)
    cfg = synth.with_histories_scaled(cfg, 400_000)
    cnt = cfg["source"]["aperture"]["counts"].astype(np.int64)
    tot = int(cnt.sum())
    eng = E.Engine(0, seed=13).configure(cfg, tally=1, batches=2, max_chunk=1 << 18)
    eng.bind()
    eng.run(tot)
    whole = eng.image()[0].cpu().numpy() * tot
    eng.reset()
    cut = int(cnt[:17].sum())
    eng.run(cut)
    eng.run(tot - cut, first=cut)
    parts = eng.image()[0].cpu().numpy() * tot
    assert whole.sum() > 0
    np.testing.assert_array_equal(parts, whole)


def test_full_size_coupled_runs(E):
    """The full 256x256x128 / 1024x768 workload runs in large chunks without device errors
    and gives a finite, non-trivial image."""
    cfg = synth.coupled_hetero()
    eng = E.Engine(0, seed=3).configure(cfg, batches=64, max_chunk=1 << 24)
    eng.bind()
    eng.run(40_000_000)
    m, v = eng.image()
    m = m.cpu().numpy()
    assert bool(np.isfinite(m).all()) and m.max() > 0
    c = eng.counters()
    assert c["error_word"] == 0 and c["tally_deposits"] > 0
    # the open field (15x15 cm at the phosphor) is brighter than the region outside it
    inner = m[512 - 64:512 + 64, 384 - 64:384 + 64].mean()
    outer = m[:100, :100].mean()
    assert inner > 5 * outer


def test_sigma_bar_falls_as_inverse_sqrt_n(E):
    """The per-pixel relative uncertainty over the bright pixels falls as 1/sqrt(N).  One pixel
    set serves both stages: the pixels at >= 50% of the final (4x less noisy) image's maximum;
    selecting at each stage by its own noisy maximum would favour the brightest pixels early
    and bias the ratio.  The engine's sigma-bar is the same statistic on its own selection."""
    cfg = synth.coupled_hetero_small()
    eng = E.Engine(0, seed=3).configure(cfg, batches=64, max_chunk=1 << 24)
    eng.bind()
    eng.run(40_000_000)
    m1, v1 = (t.cpu().numpy() for t in eng.image())
    eng.run(120_000_000, first=40_000_000)
    m2, v2 = (t.cpu().numpy() for t in eng.image())
    sel = m2 >= 0.5 * m2.max()
    s1 = float(np.mean(np.sqrt(v1[sel]) / m1[sel]))
    s2 = float(np.mean(np.sqrt(v2[sel]) / m2[sel]))
    print("sigma-bar on a fixed pixel set:", s1, s2, "ratio", s2 / s1)
    assert s1 < 0.2
    assert s2 == pytest.approx(s1 / 2.0, rel=0.05)
    assert eng.sigma_bar(0.5) == pytest.approx(sigma_bar(m2, v2, 0.5), rel=1e-9)


def test_history_ids_beyond_2_32(E, orc):
    """History ids are 64-bit: a run across 2^32 equals the runs on either side of it (fixed
    point: exactly), the block above 2^32 draws different streams from the block below, and
    histories from id 5e9 pass the same z-gate against the oracle as histories from id 0."""
    cfg = synth.coupled_hetero_small()
    b = 1 << 32
    eng = E.Engine(0, seed=11).configure(cfg, tally=1, batches=2, max_chunk=1 << 16)
    eng.bind()
    eng.run(300_000, first=b - 100_000)
    across = eng.image()[0].cpu().numpy()
    eng.reset()
    eng.run(100_000, first=b - 100_000)
    eng.run(200_000, first=b)
    split = eng.image()[0].cpu().numpy()
    assert across.sum() > 0
    np.testing.assert_array_equal(across, split)
    eng.reset()
    eng.run(200_000, first=0)
    low = eng.image()[0].cpu().numpy()
    eng.reset()
    eng.run(200_000, first=b)
    high = eng.image()[0].cpu().numpy()
    assert not np.array_equal(low, high)

    cfg = synth.kerma_water()
    om, ov, *_ = oracle_image(orc, "kerma_water", cfg, 8_000_000)
    eng = E.Engine(0, seed=1).configure(cfg, batches=64, max_chunk=1 << 24)
    eng.bind()
    eng.run(80_000_000, first=5_000_000_000)
    gm, gv = (t.cpu().numpy() for t in eng.image())
    g = z_gate(gm, gv, om, ov, thr=0.10, k=4)
    print("kerma_water z-gate, ids from 5e9", g)
    assert g["ok"], g


def test_run_until_stops_at_target(E):
    cfg = synth.kerma_water(npx=16, pitch=1.6)
    eng = E.Engine(0, seed=4).configure(cfg, batches=64, max_chunk=1 << 22)
    eng.bind()
    done, sb = eng.run_until(0.05, thr=0.5, step=2_000_000, max_hist=200_000_000)
    assert sb <= 0.05 and done <= 200_000_000
    assert eng.sigma_bar(0.5) == pytest.approx(sb)


def test_run_until_repeats_a_segmented_field(E):
    """run_until on a segmented field steps whole deliveries, with history ids continuing
    past the field's total (new, independent deliveries), until sigma-bar reaches half of one
    delivery's: it stops on a whole number of deliveries, at least 2 and no more than the 1/N
    law with the selection bias of a noisy first image allows."""
    cfg = synth.imrt_field(shape=(64, 64, 32), spacing=0.8, npx=(48, 64), pitch=0.624)
    cfg = synth.with_histories_scaled(cfg, 500_000)
    tot = int(cfg["source"]["aperture"]["counts"].sum())
    eng = E.Engine(0, seed=23).configure(cfg, tally=1, batches=16, max_chunk=1 << 19)
    eng.bind()
    eng.run(tot)
    sb1 = eng.sigma_bar(0.5)
    eng.reset()
    done, sb = eng.run_until(0.5 * sb1, thr=0.5, first=0, step=tot, max_hist=40 * tot)
    print("one delivery", sb1, "run-until", done // tot, "deliveries, sigma-bar", sb)
    assert sb <= 0.5 * sb1 and done % tot == 0 and 2 <= done // tot < 40
    assert eng.sigma_bar(0.5) == pytest.approx(sb)


def test_kahan_mode_at_the_benchmark_size(E):
    """The Kahan tally on the full coupled workload (1024 x 768 pixels of 0.39 mm, 2e7
    histories in one chunk) gives the FP64 tally's image to FP32 rounding."""
    cfg = synth.coupled_hetero()
    m0, _, _ = gpu_image(E, cfg, 20_000_000, seed=29, tally=0, batches=8, max_chunk=1 << 25)
    m2, _, eng = gpu_image(E, cfg, 20_000_000, seed=29, tally=2, batches=8, max_chunk=1 << 25)
    assert m0.sum() > 0 and eng.counters()["error_word"] == 0
    np.testing.assert_allclose(m2, m0, rtol=2e-6, atol=1e-13)


def test_autotuner_times_the_candidates_that_fit(E):
    from paper_2510_24154_amd.autotune import tune_chunk
    cfg = synth.coupled_hetero_small()
    best, rates = tune_chunk(cfg, 2_000_000, candidates=(1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 26))
    print("autotune:", rates, "best", best)
    assert best in rates and rates[best] == max(rates.values())
    assert set(rates) >= {1 << 16, 1 << 18, 1 << 20}
    assert (1 << 26) not in rates   # more than twice the histories per run
    assert all(v > 0 for v in rates.values())


def test_segmented_field_beyond_2_32_histories(E):
    """A field whose segment counts sum past 2^32: histories from id 2^32 fall in the second
    segment, so they give exactly (fixed point) the image of a one-segment field with that
    segment's aperture over the same ids."""
    cfg = synth.coupled_hetero_small()
    ap = cfg["source"]["aperture"]
    n_pairs = ap["a"].shape[1]
    a2, b2 = ap["a"].copy(), ap["b"].copy()
    a2[0, : n_pairs // 2] = 0.0          # the second segment: the field's lower half only
    b2[0, : n_pairs // 2] = 0.0
    two = copy.deepcopy(cfg)
    two["source"]["aperture"] = dict(ap, a=np.concatenate([ap["a"], a2]), b=np.concatenate([ap["b"], b2]),
                                     counts=np.array([1 << 32, 300_000], np.uint64))
    one = copy.deepcopy(cfg)
    one["source"]["aperture"] = dict(ap, a=a2, b=b2, counts=np.array([0], np.uint64))
    imgs = []
    for c in (two, one):
        eng = E.Engine(0, seed=17).configure(c, tally=1, batches=4, max_chunk=1 << 17)
        eng.bind()
        eng.run(300_000, first=1 << 32)
        imgs.append(eng.image()[0].cpu().numpy())
    assert imgs[0].sum() > 0
    np.testing.assert_array_equal(imgs[0], imgs[1])


def test_ids_past_the_total_deliver_the_field_again(E):
    """Ids past a segmented field's total T repeat the delivery: id h samples the segment of
    h mod T with its own random stream.  Exactly (fixed point): ids from T + c0 give the image
    of a one-segment field with the second segment's aperture over the same ids, ids from 2T
    that of the first segment's; the field's ids [0, 2T) in one call give the image of two
    calls, one per delivery; and the second delivery is not a copy of the first."""
    cfg = synth.coupled_hetero_small()
    ap = cfg["source"]["aperture"]
    n_pairs = ap["a"].shape[1]
    a2, b2 = ap["a"].copy(), ap["b"].copy()
    a2[0, : n_pairs // 2] = 0.0          # the second segment: the field's lower half only
    b2[0, : n_pairs // 2] = 0.0
    c0, c1 = 200_000, 100_000
    T = c0 + c1
    two = copy.deepcopy(cfg)
    two["source"]["aperture"] = dict(ap, a=np.concatenate([ap["a"], a2]), b=np.concatenate([ap["b"], b2]),
                                     counts=np.array([c0, c1], np.uint64))

    def single(a, b):
        c = copy.deepcopy(cfg)
        c["source"]["aperture"] = dict(ap, a=a, b=b, counts=np.array([0], np.uint64))
        return c

    def image(c, runs, batches=4):
        eng = E.Engine(0, seed=19).configure(c, tally=1, batches=batches, max_chunk=1 << 17)
        eng.bind()
        for first, n in runs:
            eng.run(n, first=first)
        return eng.image()[0].cpu().numpy()

    n = 50_000
    m = image(two, [(T + c0, n)])
    assert m.sum() > 0
    np.testing.assert_array_equal(m, image(single(a2, b2), [(T + c0, n)]))
    np.testing.assert_array_equal(image(two, [(2 * T, n)]), image(single(ap["a"], ap["b"]), [(2 * T, n)]))
    whole = image(two, [(0, 2 * T)])
    np.testing.assert_array_equal(whole, image(two, [(0, T), (T, T)]))
    d1, d2 = image(two, [(0, T)]), image(two, [(T, T)])
    assert not np.array_equal(d1, d2)
    assert abs(d2.sum() / d1.sum() - 1.0) < 0.05


def test_bench_configuration_energy_ledger(E):
    """The benchmark's launch configuration: the full coupled workload, 1e8 histories as one
    2^27-history chunk, 64 batches, host-driven passes with 4 items per lane (the launch
    tuner's pick), with the per-history energy ledger on: every history closes to 1e-9 and
    the image is finite."""
    cfg = synth.coupled_hetero()
    eng = E.Engine(0, seed=1).configure(cfg, batches=64, max_chunk=1 << 27, diag=True)
    eng.bind()
    eng.set_passes(0, 4)
    eng.run(100_000_000)
    c = eng.counters()
    print("bench configuration: ledger", c["max_ledger_resid"], "woodcock/history", c["woodcock_steps"] / 1e8)
    assert c["error_word"] == 0 and c["max_ledger_resid"] < 1e-9
    assert c["e_deposited"] == pytest.approx(c["e_in"], rel=1e-12)
    m, v = eng.image()
    assert bool(np.isfinite(m.cpu().numpy()).all()) and float(m.sum()) > 0


def test_kahan_mode_is_reproducible(E):
    """The Kahan tally reduces each pixel's records in a canonical order (ascending value), so
    a repeated run with the same seed and chunk size gives the same image bit for bit."""
    cfg = synth.coupled_hetero_small()
    m0, v0, _ = gpu_image(E, cfg, 400_000, seed=11, tally=2, max_chunk=1 << 16)
    m1, v1, _ = gpu_image(E, cfg, 400_000, seed=11, tally=2, max_chunk=1 << 16)
    assert m0.sum() > 0
    assert np.array_equal(m0, m1) and np.array_equal(v0, v1)


def test_kahan_image_is_the_exact_sum_of_its_records(E):
    """The Kahan tally's workgroup reduction (compensated FP32 partials per slice of 8 records,
    added per element in slice order) against the exact FP64 sum of the same records.  A
    narrow field on 0.39 mm pixels puts several LDS chunks of records into one tile of 256
    elements and tens of records into one element, so element runs cross slices and chunks.
    Compensated sums of positive terms stay within a few FP32 units of the exact sum."""
    cfg = synth.narrow_field(field=1.0, npx=64)
    n, B = 4_000_000, 2
    m, _, eng = gpu_image(E, cfg, n, seed=31, tally=2, batches=B, max_chunk=1 << 22)
    pix, e, nrec = eng.debug_records(1 << 22)
    assert nrec == len(pix) > 10_000
    npix = m.size
    pix = pix.astype(np.int64)
    exact = np.zeros(B * npix)
    np.add.at(exact, pix, e.astype(np.float64))
    cnt = np.bincount(pix, minlength=B * npix)
    print("records", nrec, "max per element", int(cnt.max()), "max per tile",
          int(np.add.reduceat(cnt, np.arange(0, B * npix, 256)).max()))
    assert np.add.reduceat(cnt, np.arange(0, B * npix, 256)).max() > 2 * 2048
    assert cnt.max() > 32
    want = exact.reshape(B, npix).sum(axis=0) / n
    np.testing.assert_allclose(m.reshape(-1), want, rtol=1e-6, atol=0)


@pytest.mark.parametrize("case", ["tiny_grid", "coupled_small"])
def test_fixed_point_image_is_the_rebinned_deposit_records(E, case):
    """Brute force on the device: the same seed gives the same trajectories in every tally
    mode, so the Kahan mode's raw deposit records, quantised to 2^-32 MeV (round half to even)
    and added per variance batch and pixel on the host, give the fixed-point mode's image
    exactly, and its batch variance to rounding: no deposit lost, duplicated or misplaced."""
    from tests._oracle_pins import tiny_grid
    cfg = tiny_grid() if case == "tiny_grid" else synth.coupled_hetero_small()
    n, B = 200_000, 16
    m1, v1, _ = gpu_image(E, cfg, n, seed=21, tally=1, batches=B, max_chunk=1 << 18)
    _, _, eng = gpu_image(E, cfg, n, seed=21, tally=2, batches=B, max_chunk=1 << 18)
    pix, e, nrec = eng.debug_records(1 << 21)
    assert nrec == len(pix) > 1000
    npix = m1.size
    assert int(pix.max()) < B * npix
    q = np.rint(e.astype(np.float64) * 2.0 ** 32).astype(np.int64)
    acc = np.zeros(B * npix, dtype=np.int64)
    np.add.at(acc, pix.astype(np.int64), q)
    s = np.zeros(npix)
    s2 = np.zeros(npix)
    for b in range(B):
        nb = (-(-(b + 1) * n // B)) - (-(-b * n // B))
        v = acc[b * npix:(b + 1) * npix].astype(np.float64) * 2.0 ** -32
        s = s + v
        s2 = s2 + v * v / nb
    assert np.array_equal(s / n, m1.reshape(-1))
    var = np.maximum((s2 - s * s / n) / (n * (B - 1)), 0.0)
    np.testing.assert_allclose(var, v1.reshape(-1), rtol=1e-9, atol=0)
