"""Host logic of the benchmark (no GPU): the one-GPU refusal and the roofline arithmetic of the
dominant kernel, checked against the per-stage byte counts written out by hand."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_stage_byte_counts():
    # factor: H (17 x 17 upper triangle, 153 words), G (13 x 17), Delta (13), right-hand side (30) read;
    # L_u (10), K (4 x 13), S (13 x 13 upper triangle, 91), affine terms (17) written
    assert bench.FACTOR_WORDS_PER_STAGE == 153 + 221 + 13 + 30 + 10 + 52 + 91 + 17
    assert 8 * bench.FACTOR_WORDS_PER_STAGE == 4696
    assert 8 * bench.SOLVE_WORDS_PER_STAGE == 3608


def test_async_kernel_roofline_from_counts_and_time():
    w = types.SimpleNamespace(N=30)
    st = dict(factorizations=1000, fused_factorizations=1000, solves=1200, fused_solves=1200)
    kt = {"async": (500.0, 4), "setup": (0.1, 1)}
    dom, out = bench.kernel_roofline(w, st, kt)
    assert dom == "k_run"
    r = out["k_run"]
    per_launch = (1000 * 31 * 4696 + 1200 * 31 * 3608) / 4
    assert r["bytes_per_launch"] == pytest.approx(per_launch)
    assert r["avg_ms"] == pytest.approx(125.0)
    assert r["achieved"] == pytest.approx(per_launch / 0.125 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    # FP32 factor words are half as wide
    _, out32 = bench.kernel_roofline(w, st, kt, word_bytes=4.0)
    assert out32["k_run"]["bytes_per_launch"] == pytest.approx(per_launch / 2)
