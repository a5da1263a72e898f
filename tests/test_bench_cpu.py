"""Host logic of bench.py: the roofline object and the one-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(dominant, ms=10.0, launches=4, work=4.0e12):
    """A run record whose class `dominant` has the most GPU time."""
    n = len(bench.CLASSES)
    r = {"ms": [1.0] * n, "launches": [1] * n, "work": [1.0] * n}
    i = bench.CLASSES.index(dominant)
    r["ms"][i], r["launches"][i], r["work"][i] = ms, launches, work
    return r


def test_roofline_bound_and_units_per_class():
    # 4 launches of 1e12 units in 10 ms: 2.5 ms per launch
    hbm = bench.roofline_for(_run("plane"), "c2")
    assert hbm["bound"] == "hbm" and hbm["unit"] == "GB/s" and hbm["peak"] == 8000.0
    assert hbm["achieved"] == pytest.approx(1e12 / 2.5e-3 / 1e9)
    mm = bench.roofline_for(_run("rotate"), "c2")
    assert mm["bound"] == "mfma" and mm["unit"] == "TFLOP/s" and mm["peak"] == 78.6
    assert mm["achieved"] == pytest.approx(1e12 / 2.5e-3 / 1e12)
    alu = bench.roofline_for(_run("rayleigh_ritz"), "c2")
    assert alu["bound"] == "alu" and alu["symbol"] == "k_rr_lds"
    for rf in (hbm, mm, alu):
        assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-4)
        assert rf["avg_launch_us"] == pytest.approx(2500.0)
        assert rf["launches"] == 4


def test_traffic_only_for_the_counted_source_and_workload(monkeypatch):
    # counters taken on the source as it is now
    fresh = {k: dict(v, sha256=bench.source_sha(v["source"])) for k, v in bench.PMC_TRAFFIC.items()}
    monkeypatch.setattr(bench, "PMC_TRAFFIC", fresh)
    for name, t in fresh.items():
        assert bench.roofline_for(_run(name), t["config"])["traffic"] == t["bytes_per_launch"]
        assert bench.roofline_for(_run(name), "c3")["traffic"] is None
        assert bench.roofline_for(_run(name), t["config"], with_traffic=False)["traffic"] is None
    # a changed source voids the counters
    stale = {k: dict(v, sha256="0" * 64) for k, v in bench.PMC_TRAFFIC.items()}
    monkeypatch.setattr(bench, "PMC_TRAFFIC", stale)
    for name, t in stale.items():
        assert bench.roofline_for(_run(name), t["config"])["traffic"] is None
    # classes without counters report none
    assert bench.roofline_for(_run("nonlocal"), "c2")["traffic"] is None


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
    with pytest.raises(json.JSONDecodeError):
        json.loads(p.stdout or "x")


def test_hpsi_rates_use_the_per_state_count_and_the_pass_bytes():
    """The algorithmic H*psi rate divides the per-state count (2Ns + Ns/J + nnz(s+4)/J,
    summed by the library) by the three H*psi classes' time; the pass rate their own
    bytes by the same time; a run without H*psi time reports none."""
    n = len(bench.CLASSES)
    r = {"ms": [2.0, 1.0, 1.0] + [5.0] * (n - 3), "work": [1e9, 2e9, 1e9] + [7.0] * (n - 3),
         "hpsi_alg_bytes": 2e9}
    alg, passes = bench.hpsi_rates(r)
    assert alg == pytest.approx(2e9 / 4e-3 / 1e9, rel=1e-3)
    assert passes == pytest.approx(4e9 / 4e-3 / 1e9, rel=1e-3)
    r0 = dict(r, ms=[0.0, 0.0, 0.0] + [5.0] * (n - 3))
    assert bench.hpsi_rates(r0) == (None, None)


def test_inner_scf_correction_is_smooth_and_decays():
    import numpy as np
    import workloads as W
    el = W.small_slab(n_states=8)[0]
    d = bench.smooth_field(el, 3, 0.05)
    assert d.shape == (el.npts,) and np.max(np.abs(d)) <= 0.05 + 1e-15
    # one cosine per axis: the 3D DFT has 8 nonzero coefficients (+-1 per axis)
    F = np.fft.fftn(d.reshape(el.n[2], el.n[1], el.n[0]))
    assert np.sum(np.abs(F) > 1e-9 * np.abs(F).max()) == 8
