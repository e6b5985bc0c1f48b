"""Host-side checks of bench.py's contract helpers (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_counts_algorithmic_flops_of_the_dominant_family():
    import bench
    n, p = 1000, 1000
    # family: (launches, ms, active node-iterations)
    prof = {"gemm_xw.f32": (10, 0.10, 2560), "admm_xtu.f32": (10, 0.12, 2560), "gap_check": (2, 0.05, 0)}
    roof, kernels = bench.roofline(prof, n, p)
    assert roof["kernel"] == "admm_xtu.f32"
    achieved = 2.0 * n * p * 2560 / (0.12e-3) / 1e12
    assert roof["achieved"] == pytest.approx(achieved, rel=1e-3)
    assert roof["peak"] == 157.3 and roof["frac"] == pytest.approx(achieved / 157.3, rel=1e-3)
    assert roof["traffic"] is None          # not asked for
    assert set(kernels) == set(prof)


def test_counter_traffic_is_dropped_when_the_kernel_sources_change(tmp_path, monkeypatch):
    import bench
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    (prof_dir / bench.TRAFFIC_FILE).write_text(json.dumps(
        {"c3": {"source_digest": "not-the-current-sources", "per_launch_bytes": {"admm_xtu.bf16": 123}}}))
    csrc = tmp_path / "paper_2602_04551_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("__global__ void k() {}\n")
    (csrc / "b.hpp").write_text("// header\n")
    (csrc / "host.hip").write_text("// host code only\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("admm_xtu.bf16", "c3") is None
    import hashlib
    digest = hashlib.sha256(b"__global__ void k() {}\n// header\n").hexdigest()
    (prof_dir / bench.TRAFFIC_FILE).write_text(json.dumps(
        {"c3": {"source_digest": digest, "per_launch_bytes": {"admm_xtu.bf16": 123}}}))
    assert bench.measured_traffic("admm_xtu.bf16", "c3") == 123
    assert bench.measured_traffic("admm_xtu.bf16", "c5") is None     # no counters for that workload
    # a host-only file may change; a kernel file or a header may not
    (csrc / "host.hip").write_text("// host code, edited\n")
    assert bench.measured_traffic("admm_xtu.bf16", "c3") == 123
    (csrc / "b.hpp").write_text("// header, edited\n")
    assert bench.measured_traffic("admm_xtu.bf16", "c3") is None


def test_sweep_bytes_roofline_counts_operand_and_state_bytes():
    """HBM view of the node-batch sweeps: per sweep the stored operand twice
    (2 n p b_X, b_X = 1 for FP8 codes) plus 16 p + p / 4 bytes per active node,
    over the summed time of both contractions."""
    import bench
    n, p = 1000, 50000
    prof = {"gemm_xw.fp8": (100, 40.0, 25600), "admm_xtu.fp8": (100, 60.0, 25600)}
    r = bench.sweep_bytes_roofline(prof, n, p, "fp8")
    nbytes = 100 * 2.0 * n * p * 1 + 25600 * (16.0 * p + p / 4.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(nbytes / 0.1 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert bench.sweep_bytes_roofline({}, n, p, "fp32") is None
