"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the roofline
arithmetic and the guard that ties counter summaries to the kernel sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_corr_roofline_fractions():
    r = bench.corr_roofline("fp32", flops=1.573e11, corr_ms=2.0, traffic=None, transforms=10)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(78.65, rel=1e-3)
    assert r["frac"] == pytest.approx(0.5, rel=1e-3)
    assert "mfma_issued_frac" not in r
    # exact-length mode: against the FP16 matrix peak, with the issued matrix-core flops beside it
    n = 500000  # fractions are reported to four decimals
    x = bench.corr_roofline("fp16pfa", flops=1e12, corr_ms=1.0, traffic=1e9, transforms=n)
    assert x["bound"] == "mfma" and x["peak"] == bench.PEAK_MFMA_F16_TFLOPS
    assert x["frac"] == pytest.approx(1e12 / 1e-3 / 1e12 / 2500.0, abs=1e-4)
    assert x["mfma_flops_issued_per_launch"] == n * 54 * 16384
    assert x["mfma_issued_frac"] == pytest.approx(n * 54 * 16384 / 1e-3 / 1e12 / 2500.0, abs=1e-4)
    assert x["traffic"] == 1e9


def test_traffic_only_from_summaries_of_the_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc123def456")
    assert bench.read_traffic("corr", "weak") is None  # no summary
    (prof / "corr_weak_counters.md").write_text("hbm_bytes_per_launch: 1.5e+09\n\nsource_hash: abc123def456\n")
    assert bench.read_traffic("corr", "weak") == pytest.approx(1.5e9)
    (prof / "corr_weak_counters.md").write_text("hbm_bytes_per_launch: 1.5e+09\n\nsource_hash: 000000000000\n")
    assert bench.read_traffic("corr", "weak") is None  # taken on other sources
