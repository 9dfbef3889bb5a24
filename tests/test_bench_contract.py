"""Host-side checks of bench.py (no GPU): the one-GPU contract and the rate
arithmetic of its kernel summaries."""
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


def test_kernel_rates():
    st = {"far32_launches": 4, "far32_ms": 30.0, "far32_flops": 5.0e11,
          "mixed64_launches": 4, "mixed64_ms": 4.0, "mixed64_flops": 3.0e10,
          "direct_launches": 0, "direct_ms": 0.0, "direct_flops": 0.0}
    out = bench.mixed_kernel_rates(st)
    assert set(out) == {"far32", "mixed64"}
    far = out["far32"]
    assert far["avg_launch_ms"] == pytest.approx(7.5)
    assert far["achieved"] == pytest.approx(5.0e11 / 7.5e-3 / 1e12)
    assert far["frac"] == pytest.approx(far["achieved"] / bench.PEAK_FP32_VALU_TFLOPS)
    assert out["mixed64"]["peak"] == bench.PEAK_FP64_VALU_TFLOPS
    st.update(eq_launches=2, eq_far_ms=8.0, eq_far_flops=1.0e11, eq_near_ms=1.0, eq_near_flops=1.0e10)
    out = bench.mixed_kernel_rates(st)
    assert set(out) == {"far32", "mixed64", "eq_far", "eq_near"}
    assert out["eq_far"]["avg_launch_ms"] == pytest.approx(4.0)
    assert out["eq_far"]["peak"] == bench.PEAK_FP32_VALU_TFLOPS
    assert out["eq_near"]["peak"] == bench.PEAK_FP64_VALU_TFLOPS


def test_traffic_constant_matches_counter_summary():
    """The HBM traffic reported for the direct sum comes from the committed
    rocprofv3 counter summary of the headline workload (FETCH_SIZE x 2 +
    WRITE_SIZE, KiB); without such a summary it is reported as null."""
    path = os.path.join(ROOT, "profiles", "k_direct_f64_packing2000_fp64_hbm_counters.md")
    if bench.DIRECT_TRAFFIC_BYTES is None:
        assert not os.path.exists(path)
        return
    row = next(l for l in open(path) if l.startswith("| `k_direct_f64<2, false>`"))
    fetch, write = (float(c.replace(" ", "")) for c in row.split("|")[2:4])
    assert bench.DIRECT_TRAFFIC_BYTES == pytest.approx((2 * fetch + write) * 1024, rel=1e-5)


def test_offdiag_error_ignores_identity_part():
    mu = np.array([1e6, -2e6, 3.0, 4.0])
    ref = mu + np.array([1.0, 2.0, -4.0, 0.5])
    y = ref + np.array([0.0, 0.0, 4e-3, 0.0])
    assert bench.offdiag_err(y, ref, mu) == pytest.approx(1e-3)


def test_budget():
    b = bench.Budget(100.0)
    assert b.fits(50.0) and not b.fits(150.0)


def test_serve_only_needs_requests():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--serve-only", "--serve-requests", "0"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "--serve-requests" in r.stderr
    assert r.stdout.strip() == ""


def test_profile_summaries_are_short_text_with_their_command():
    """profiles/ holds short rocprofv3 summaries as text: each names the
    kernel and workload in its file name, gives the full command, which runs
    committed files only (the benchmark), and is a few KB."""
    pdir = os.path.join(ROOT, "profiles")
    names = sorted(os.listdir(pdir))
    assert names
    for n in names:
        assert n.endswith((".md", ".txt")) and n.startswith("k_"), n
        text = open(os.path.join(pdir, n)).read()
        assert len(text.encode()) < 16384, n
        cmd = [l for l in text.splitlines() if "rocprofv3" in l and "--" in l]
        assert cmd, n
        for l in cmd:
            assert "bench.py" in l and "_work" not in l, (n, l)
