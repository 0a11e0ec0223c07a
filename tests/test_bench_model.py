"""The measurement model of bench.py (CPU only): algorithmic flops and bytes per
launch of each kernel kind, the roofline bound chosen by arithmetic intensity,
the counter table gated on the kernel sources' digest, and the refusal of more
than one GPU.  The figures are the ones the roofline object of the bench line
divides by the measured launch durations."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

P, N1 = 64, 512
N = P * N1 * N1  # elements of a 512 x 512 x 64 tensor


def test_slice_gemm_work():
    # p products of 512 x 512 by 512 x 512 (Algorithm 1 step 2): A~ read, X~ read, C~ written
    f, b = bench.kernel_work("gemm", P, N1, N1, N1, 4)
    assert f == 2.0 * 512 ** 3 * 64 == 17179869184.0
    assert b == 4 * N + 4 * N + 4 * N
    f2, b2 = bench.kernel_work("gemm", P, N1, N1, N1, 2)
    assert f2 == f and b2 == 2 * N + 2 * N + 4 * N   # 16-bit operands, FP32 products


def test_transform_work_by_launch_mix():
    # dense p x p per tube: 2p flops per element
    f, _ = bench.kernel_work("tube_inv", P, N1, N1, N1, 4, per_solve=1)
    assert f == 2.0 * P * N
    # the only inverse of a paired solve is that of M*(C): no src
    assert bench.kernel_work("tube_inv", P, N1, N1, N1, 4, per_solve=1)[1] == 8 * N
    # 2k + 1 inverses per unpaired solve, all but M*(C)'s with a src
    k = 40
    b = bench.kernel_work("tube_inv", P, N1, N1, N1, 4, per_solve=2 * k + 1)[1]
    assert b == pytest.approx(8 * N + 4 * N * 2 * k / (2 * k + 1))
    # forward: input read, X~ written in the GEMM type; M*(C)'s also writes U_1 (FP32)
    assert bench.kernel_work("tube_fwd", P, N1, N1, N1, 2, per_solve=2)[1] == 4 * N + 2 * N + 2 * N
    assert bench.kernel_work("tube_fwd", P, N1, N1, N1, 4, per_solve=2)[1] == 4 * N + 4 * N + 2 * N
    # paired transforms: two transforms; products and src read, y (FP32) and X~ written
    f, b = bench.kernel_work("tube_pair", P, N1, N1, N1, 2)
    assert f == 4.0 * P * N and b == (12 + 2) * N


def test_fast_transform_flops():
    # O(p log p): 5 log2(p) flops per element for long tubes
    p = 256
    f, b = bench.kernel_work("tube_fwd", p, 256, 256, 256, 4, fast=True, per_solve=81)
    assert f == pytest.approx(5.0 * 8 * p * 256 * 256)
    assert b == pytest.approx(8.0 * p * 256 * 256 + 4.0 * p * 256 * 256 / 81)


def test_roofline_bound_by_intensity():
    # FP32 GEMM: 85 flop/B, above the FP32 ridge 157.3e12 / 8e12 = 19.7: MFMA-bound
    f, b = bench.kernel_work("gemm", P, N1, N1, N1, 4)
    r = bench.roofline_entry("gemm", 140.0, f, b, "f32")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(f / 140e-6 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    # BF16 GEMM: 128 flop/B, below the BF16 ridge 2500e12 / 8e12 = 312.5: HBM-bound
    f, b = bench.kernel_work("gemm", P, N1, N1, N1, 2)
    r = bench.roofline_entry("gemm", 40.0, f, b, "bf16")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(b / 40e-6 / 1e9)
    # transforms are priced against FP32 arithmetic whatever the GEMM type
    f, b = bench.kernel_work("tube_pair", P, N1, N1, N1, 2)
    r = bench.roofline_entry("tube_pair", 60.0, f, b, "bf16")
    assert r["bound"] == "hbm" and r["arith_intensity"] == pytest.approx(4.0 * P / 14)


def test_counter_tables_follow_the_sources(monkeypatch):
    # the stored HBM bytes are reported only while the kernel sources hash to the
    # digest the counters were taken from
    assert bench.hyper_traffic("gemm", "f32") == bench.HYPER_TRAFFIC["bytes"]["f32/gemm"]
    assert bench.hyper_traffic("tube_inv", "f32") is None   # no counter entry for it
    monkeypatch.setitem(bench.HYPER_TRAFFIC, "digest", "0" * 16)
    assert bench.hyper_traffic("gemm", "f32") is None
    assert bench.measured_traffic("fused_fwd", "f32") == bench.TRAFFIC["bytes"]["fused_fwd"]
    assert bench.measured_traffic("fused_fwd", "bf16") is None
    monkeypatch.setitem(bench.TRAFFIC, "digest", "0" * 16)
    assert bench.measured_traffic("fused_fwd", "f32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
