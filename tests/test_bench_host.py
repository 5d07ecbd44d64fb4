"""Host logic of bench.py (no GPU): the one-GPU contract, the roofline arithmetic,
and the HBM-traffic lookup that must go null when a kernel's source changes."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_direct_and_mfma():
    """The dominant kernel (largest timed total) and its algorithmic rate from the
    library's work count: 2 flop per tone-sample on the direct kernels over the
    FP32 vector peak, 4 on the angle-addition products over the matrix peak."""
    K, L = 1000, 1 << 24
    stats = {"direct_kernel": (5, 5 * 2.0, 2.1, 5.0 * K * L)}         # 2 ms per launch
    r = bench.roofline_for(stats)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP32_TFLOPS
    assert abs(r["achieved"] - 2.0 * K * L / 2e-3 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert r["work_per_launch"] == K * L
    stats = {"angle_gemm_kernel_bf16": (5, 5 * 0.16, 0.17, 5.0 * K * L), "gen_a_kernel_bf16": (5, 5 * 0.013, 0.02, 0.0)}
    r = bench.roofline_for(stats)
    assert r["bound"] == "mfma" and r["kernel"] == "angle_gemm_kernel_bf16"
    assert abs(r["achieved"] - 4.0 * K * L / 0.16e-3 / 1e12) < 1e-6
    assert abs(r["issued_tflops_min"] - 3 * r["achieved"]) < 1e-6 and r["peak"] == bench.PEAK_MFMA16_TFLOPS
    # the hybrid product counts only the tone-samples it covers
    stats = {"hyb_gemm_bf16": (4, 4 * 0.1, 0.11, 4 * 9900.0 * (1 << 20)),
             "direct_hybrid_kernel": (4, 4 * 0.05, 0.06, 4 * 100.0 * (1 << 20))}
    r = bench.roofline_for(stats)
    assert r["kernel"] == "hyb_gemm_bf16" and abs(r["achieved"] - 4.0 * 9900 * (1 << 20) / 0.1e-3 / 1e12) < 1e-6


def test_traffic_lookup_follows_the_source_hash(tmp_path, monkeypatch):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, v in rec.items():
        if key.startswith("_"):
            continue
        src = open(os.path.join(ROOT, v["source"]), "rb").read()
        ok = hashlib.sha256(src).hexdigest()[:16] == v["sha256_16"]
        assert bench.traffic_for(key) == (v["bytes_per_launch"] if ok else None)
        # the KiB figures are stored to 0.1 KiB, the byte count from the unrounded ones
        assert abs(v["bytes_per_launch"] - (v["fetch_kib"] * v["fetch_scale"] +
                                            v["write_kib"] * v["write_scale"]) * 1024) < 256
    # a stale hash gives null, an unknown kernel too
    fake = tmp_path / "repo"
    (fake / "profiles").mkdir(parents=True)
    (fake / "k.hip").write_text("kernel")
    (fake / "profiles" / "traffic.json").write_text(json.dumps(
        {"k": {"source": "k.hip", "sha256_16": "0" * 16, "bytes_per_launch": 5}}))
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.traffic_for("k") is None
    assert bench.traffic_for("other") is None
    good = hashlib.sha256(b"kernel").hexdigest()[:16]
    (fake / "profiles" / "traffic.json").write_text(json.dumps(
        {"k": {"source": "k.hip", "sha256_16": good, "bytes_per_launch": 5}}))
    assert bench.traffic_for("k") == 5
