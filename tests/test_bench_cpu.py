"""Host-side logic (no GPU needed): bench.py's one-GPU contract, its traffic
lookup keyed by the kernel sources' hash and the accuracy gate of the whole
batched workload, and the surrogate gate's spread score."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_lookup_follows_kernel_sources(tmp_path, monkeypatch):
    """A counter entry is used only while its kernel hash matches the sources."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 1.5e9, "kernel_sha": bench._kernel_sha()}
    (prof / "hv_traffic.json").write_text(json.dumps({"cfg4_hb_c128": entry,
                                                      "cfg2_hb_c128": dict(entry, kernel_sha="0" * 16)}))
    sha = bench._kernel_sha()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_kernel_sha", lambda: sha)
    assert bench._traffic("cfg4_hb", "c128") == 1.5e9
    assert bench._traffic("cfg2_hb", "c128") is None
    assert bench._traffic("cfg4", "c64") is None


def test_curve_error_floor():
    ref = np.array([1.0, 0.5, 1e-9])
    assert bench.curve_err(ref, ref) == 0.0
    # relative where |C| is large, against 1e-3 of the maximum where it is tiny
    assert bench.curve_err(ref * np.array([1.0, 1.01, 1.0]), ref) == pytest.approx(0.01)
    assert bench.curve_err(ref + np.array([0.0, 0.0, 1e-6]), ref) == pytest.approx(1e-3)


def test_whole_workload_gate_matches_curves(tmp_path):
    """cfg3_compare pairs batched and plain curves by instance index across
    several plain files and reports the worst curve."""
    rng = np.random.default_rng(3)
    C = rng.uniform(0.5, 2.0, (6, 3, 20))
    M = rng.uniform(0.5, 2.0, (6, 3, 20))
    z = np.zeros_like(C)
    np.savez(tmp_path / "b.npz", instances=np.arange(6), lnZ=z, E=z, C=C, M=M)
    Cp = C.copy()
    Cp[4, 1, 7] *= 1.0 + 2e-3  # one curve off by 2e-3 at one temperature
    np.savez(tmp_path / "p1.npz", instances=np.array([0, 1, 2]), lnZ=z[:3], E=z[:3], C=Cp[:3], M=M[:3])
    np.savez(tmp_path / "p2.npz", instances=np.array([3, 4, 5]), lnZ=z[3:], E=z[3:], C=Cp[3:], M=M[3:])
    out = bench.cfg3_compare(str(tmp_path / "b.npz"), [str(tmp_path / "p1.npz"), str(tmp_path / "p2.npz")])
    assert out["curves_compared"] == 18
    assert out["curves_C_err_above_1e-3"] == 1
    assert out["max_C_err"] == pytest.approx(2e-3 / (1 + 2e-3), rel=1e-9)
    assert out["max_M_err"] == 0.0
    assert out["C_within_1e-3"] is False


def test_surrogate_gate_spread():
    """The gate score: zero for identical members; for two members the relative
    half-difference; the floor (1e-3 of the curve's largest mean) caps it where
    the mean curve is tiny; only temperatures from t_min up count."""
    from paper_2607_25585_amd.surrogate import c_spread
    T = np.array([0.5, 1.0, 2.0, 4.0])
    a = np.array([[1.0, 2.0, 3.0, 4.0]])
    assert c_spread(np.stack([a, a, a]), T, 1.0)[0] == 0.0
    b = a * np.array([[10.0, 1.0, 1.1, 1.0]])  # differs at T = 0.5 (ignored) and T = 2
    assert c_spread(np.stack([a, b]), T, 1.0)[0] == pytest.approx(0.1 * 3.0 / 2 / (3.15))
    tiny = np.array([[1e-9, 1.0, 1.0, 1.0]])
    tiny2 = np.array([[3e-9, 1.0, 1.0, 1.0]])
    assert c_spread(np.stack([tiny, tiny2]), T, 0.1)[0] == pytest.approx(1e-9 / 1e-3)
