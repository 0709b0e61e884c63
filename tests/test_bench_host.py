"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline's choice of roof, the
per-stage algorithmic bytes and flops of the precisions and paths, and the rule that counter traffic is
reported only for the kernel source it was measured on."""
import hashlib
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_takes_the_roof_the_intensity_reaches():
    # 1 GF over 1 GB = 1 flop/B: below every MFMA ridge -> HBM roof
    r = bench.roofline({"flops": 1e9, "bytes": 1e9}, 1.0, "fp32")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1e9 / 1e-3 / 1e9) and r["frac"] == pytest.approx(1e12 / 8e12)
    # 100 flop/B: above the FP32 ridge (157.3 / 8 = 19.7) -> FP32 MFMA roof
    r = bench.roofline({"flops": 1e11, "bytes": 1e9}, 1.0, "fp32")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(157.3)
    # the same work on the 16-bit paths sits below their ridge (2.5e15 / 8e12 = 312) -> HBM
    for prec in ("fp16x3", "bf16x3"):
        assert bench.roofline({"flops": 1e11, "bytes": 1e9}, 1.0, prec)["bound"] == "hbm"
    r = bench.roofline({"flops": 1e12, "bytes": 1e9}, 1.0, "fp64")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(78.6)


def _shapes(n_cheb=128):
    cfg = types.SimpleNamespace(n_chi=256, n_R=96, n_cheb=n_cheb, n_g=10, n_s=5)
    plan = types.SimpleNamespace(rows=288, rows_pad=288, n_ell=96)
    return plan, cfg


def test_stage_work_of_the_precisions():
    plan, cfg = _shapes()
    B = 256
    w32 = bench.stage_work(plan, cfg, "fp32", B)
    w16 = bench.stage_work(plan, cfg, "fp16x3", B)
    w64 = bench.stage_work(plan, cfg, "fp64", B)
    NP, N = 256 * 96, 128
    # FP16 hi + lo move the bytes of FP32 (4 per element); with 128 nodes and 15 bins both paths
    # contract the nodal basis with P itself: no projection stage, no coefficient row scales
    assert bench.nodal_path("fp32", cfg) and bench.nodal_path("fp16x3", cfg) and bench.nodal_path("fp64", cfg)
    assert "projection" not in w16 and "projection" not in w32 and "projection" not in w64
    assert w16["contraction"]["bytes"] == w32["contraction"]["bytes"]
    assert w16["contraction"]["flops"] == w32["contraction"]["flops"]
    assert w16["r_weights"]["bytes"] == w32["r_weights"]["bytes"]
    # 20 bins: FP16X3 projects into split coefficients with a scale per coefficient row
    cfg20 = types.SimpleNamespace(n_chi=256, n_R=96, n_cheb=128, n_g=15, n_s=5)
    assert not bench.nodal_path("fp16x3", cfg20)
    v16, v32 = bench.stage_work(plan, cfg20, "fp16x3", B), bench.stage_work(plan, cfg20, "fp32", B)
    assert v16["projection"]["bytes"] == NP * (N * (4 + 4) + 4) * B and "projection" not in v32
    assert v16["r_weights"]["bytes"] - v32["r_weights"]["bytes"] == NP * 4 * B
    # contraction: 2 flops per (row, Chebyshev node, point, set), plus the R-sum's where it is
    # fused; basis read once per launch
    rows_bins = 96 * (10 + 15 + 5)
    assert w64["contraction"]["flops"] == 2.0 * 288 * N * NP * B + 2.0 * rows_bins * NP * B
    assert w32["contraction"]["flops"] == w64["contraction"]["flops"]
    assert w32["contraction"]["bytes"] > NP * 288 * N * 4
    # the FP64 weights table is 16 wide in FP64, the FP32 one 16 wide (15 bins rounded up) in FP32
    assert w64["r_weights"]["bytes"] - w32["r_weights"]["bytes"] == NP * 16 * 4 * B
    # below batch 32 the FP64 path keeps w in memory and sums it in a separate stage
    u64 = bench.stage_work(plan, cfg, "fp64", 16)
    assert "r_weights" not in u64 and u64["contraction"]["flops"] == 2.0 * 288 * N * NP * 16
    assert u64["quad_R"]["flops"] == 2.0 * rows_bins * NP * 16
    assert bench.fused_path("fp64", 16, 32) and not bench.fused_path("fp64", 17, 256)
    assert bench.fused_path("fp16x3", 20, 1) and not bench.fused_path("fp32", 20, 31)
    # the even/odd split halves the projection's products when N % 8 == 0
    plan, cfg7 = _shapes(n_cheb=100)
    cfg96 = types.SimpleNamespace(n_chi=256, n_R=96, n_cheb=120, n_g=10, n_s=5)
    assert bench.nodal_path("fp32", cfg96) and not bench.nodal_path("fp64", cfg96)
    cfg7b = types.SimpleNamespace(n_chi=256, n_R=96, n_cheb=102, n_g=10, n_s=5)
    assert not bench.nodal_path("fp32", cfg7b)
    # FP16X3 on FP32 P needs whole 16-byte granules per row, as FP32 does
    cfg20n = types.SimpleNamespace(n_chi=256, n_R=96, n_cheb=20, n_g=10, n_s=5)
    assert bench.nodal_path("fp16x3", cfg20n) and not bench.nodal_path("fp16x3", cfg7b)
    assert bench.stage_work(plan, cfg96, "fp64", B)["projection"]["flops"] * 2 == pytest.approx(
        bench.stage_work(plan, cfg7b, "fp32", B)["projection"]["flops"] * (120 / 102) ** 2)


def test_counter_traffic_only_for_the_measured_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_2410_03632_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "eval.hip").write_bytes(b"// kernel source A\n")
    sha = hashlib.sha256(b"// kernel source A\n").hexdigest()
    (tmp_path / "profiles").mkdir()
    rec = {"records": [{"kernel": "k", "source_sha256": sha, "workload": "w", "batch": 256, "precision": "fp16x3",
                        "fetch_bytes": 10, "write_bytes": 5}]}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("k", "w", 256, "fp16x3") == 15
    assert bench.counter_traffic("k", "w", 128, "fp16x3") is None
    assert bench.counter_traffic("k", "w", 256, "fp32") is None
    (src / "eval.hip").write_bytes(b"// kernel source B\n")
    assert bench.counter_traffic("k", "w", 256, "fp16x3") is None


def test_committed_traffic_records_name_existing_profiles():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert rec["records"]
    for r in rec["records"]:
        assert os.path.exists(os.path.join(ROOT, r["profile"]))
        assert r["fetch_bytes"] > 0 and r["write_bytes"] > 0
