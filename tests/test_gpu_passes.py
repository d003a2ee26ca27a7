"""Device-driven queue passes and graph runs (the batched delivery of a whole IMRT field in
one launch), through the C ABI.  Neither may change a trajectory: with the fixed-point tally
every setting gives the same image bit for bit as host-driven passes."""
import numpy as np
import pytest

from paper_2510_24154_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_24154_amd as E
    return E


def field():
    """A 40-segment field on the coarse coupled geometry, 4e5 histories over the segments."""
    cfg = synth.imrt_field(shape=(64, 64, 32), spacing=0.8, npx=(96, 128), pitch=0.312)
    cfg = synth.with_histories_scaled(cfg, 400_000)
    return cfg, int(cfg["source"]["aperture"]["counts"].sum())


def engine(E, cfg, chunk=1 << 16, seed=21):
    eng = E.Engine(0, seed=seed).configure(cfg, tally=E.TALLY_FIXED64, batches=64, max_chunk=chunk)
    eng.bind()
    return eng


def image(eng):
    m, v = eng.image()
    return m.cpu().numpy(), v.cpu().numpy()


def test_device_driven_passes_give_the_host_driven_image(E):
    cfg, n = field()
    ref = engine(E, cfg)
    ref.set_passes(0)                      # host-driven throughout
    ref.run(n)
    m0, v0 = image(ref)
    assert m0.sum() > 0
    for dp, ipl in ((0, 4), (1, 2), (3, 2), (24, 2), (-1, 2), (-1, 1), (-1, 4), (-1, 8)):
        print("device passes", dp, "items per lane", ipl, flush=True)
        eng = engine(E, cfg)
        eng.set_passes(dp, ipl)
        eng.run(n)
        if dp == -1:
            eng.reset()
            eng.run(n)                     # the second run learns its pass count from the first
        m, v = image(eng)
        assert np.array_equal(m, m0) and np.array_equal(v, v0), (dp, ipl)


def test_graph_run_equals_eager_run_on_every_replay(E):
    """The whole field (several chunks: 2^16 histories each) captured as one graph: the first
    call captures and replays it, later calls replay it; with eager runs of another engine and
    host synchronisations between the replays, every replay gives the eager image."""
    import torch
    cfg, n = field()
    eager = engine(E, cfg)
    eager.run(n)
    m0, v0 = image(eager)
    other = engine(E, cfg, seed=5)
    g = engine(E, cfg)
    g.set_graph(True)
    for rep in range(3):
        print("graph replay", rep, flush=True)
        g.reset()
        g.run(n)
        m, v = image(g)
        torch.cuda.synchronize()
        assert np.array_equal(m, m0) and np.array_equal(v, v0), rep
        other.reset()
        other.run(n // 2)
        torch.cuda.synchronize()


def test_graph_run_with_too_few_passes_is_refused(E):
    """One captured pass cannot finish a coupled run: the run reports the leftover particles
    (every kernel still ends normally) instead of returning an incomplete image as complete."""
    cfg, n = field()
    g = engine(E, cfg)
    g.set_graph(True, 1)
    with pytest.raises(E.EpidmcError) as e:
        g.run(n)
    assert e.value.code == -7   # EPIDMC_E_OVERFLOW
    # the same engine then runs correctly with enough passes
    eager = engine(E, cfg)
    eager.run(n)
    g.set_graph(True, 16)
    g.reset()
    g.run(n)
    assert np.array_equal(image(g)[0], image(eager)[0])


def test_autotuner_fits_the_chunk_model_and_times_the_launch_axes(E):
    """The tuner times three chunk sizes, fits T = a * chunks + b, predicts every size that
    fits and times each (items per lane, pass mode) pair at the chosen chunk."""
    from paper_2510_24154_amd.autotune import tune
    cfg = synth.coupled_hetero_small()
    r = tune(cfg, 1_000_000, candidates=(1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20), ipls=(1, 2), pass_modes=(0, -1))
    print("tune:", r)
    assert r["chunk"] in r["chunk_s_predicted"]
    assert len(r["chunk_s_measured"]) == 3 and set(r["chunk_s_measured"]) <= set(r["chunk_s_predicted"])
    assert r["chunk_s_predicted"][r["chunk"]] == min(r["chunk_s_predicted"].values())
    assert len(r["launch_s"]) == 4 and all(v > 0 for v in r["launch_s"].values())
    assert r["items_per_lane"] in (1, 2) and r["device_passes"] in (0, -1)
