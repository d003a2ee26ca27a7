"""CPU checks of bench.py's host logic: the equal-accuracy fit of the denoiser comparison, the
reading of profiled HBM traffic, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_equal_rmse_recovers_a_known_plain_count():
    """Plain RMSE^2 = c / N + e_ref^2 exactly: the fit returns c, e_ref^2 and the count whose
    RMSE equals the denoised one, and the speedup at the largest run's measured rate."""
    import bench
    c, e_ref2 = 4.0e5, 0.006 ** 2
    rmse = {f"plain_{n:.0e}": (c / n + e_ref2) ** 0.5 for n in bench.DN_PLAIN}
    secs = {f"plain_{bench.DN_PLAIN[-1]:.0e}": 0.5}          # 4e9 histories/s
    n_true = 1.5e8
    den = (c / n_true + e_ref2) ** 0.5
    n_eq, speedup, e2 = bench.equal_rmse(rmse, secs, den, 0.01)
    assert n_eq == pytest.approx(n_true, rel=1e-9)
    assert e2 == pytest.approx(e_ref2, rel=1e-9)
    assert speedup == pytest.approx(n_true / 4e9 / 0.01, rel=1e-9)
    # a denoised image no better than the reference's own noise has no equivalent count
    assert bench.equal_rmse(rmse, secs, 0.005, 0.01)[0] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_profiled_traffic_needs_the_current_sources_and_workload(tmp_path, monkeypatch):
    """The traffic figure comes from a profile summary only when the summary was taken on
    the current kernel sources and the same workload; otherwise the JSON line carries null."""
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text("# summary\n\n    source_sha: abc123\n    workload: coupled\n"
                               "    traffic_bytes_per_unit[k_photon_phantom]: 80.5\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "abc123")
    assert bench.profiled_traffic("k_photon_phantom", "coupled") == (80.5, "k.md")
    assert bench.profiled_traffic("k_photon_phantom", "imrt40") == (None, None)
    assert bench.profiled_traffic("k_electron<phantom>", "coupled") == (None, None)
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "def456")
    assert bench.profiled_traffic("k_photon_phantom", "coupled") == (None, None)


def test_committed_traffic_figures_are_per_step_of_one_delivery():
    """A transport step reads one voxel or table entry at a time: past the L2 that is at most a
    few 128-byte lines.  A per-step figure far above that means the counters of several
    deliveries (the time-to-1% extrapolation runs more after the timed one) were divided by the
    step counts of one."""
    import glob
    found = 0
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(f):
            key, _, val = line.strip().partition(": ")
            if key.startswith("traffic_bytes_per_unit["):
                found += 1
                assert 0.0 < float(val) <= 512.0, (os.path.basename(f), key, val)
    assert found >= 4
