"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte count of a composite launch, and the reading of the committed counter
summary (traffic is reported only for the kernel sources it was taken on)."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_composite_bytes_regular_and_compact():
    reg = types.SimpleNamespace(offset=None)
    cmp_ = types.SimpleNamespace(offset=object())
    P, N = 1000, 20
    # 3 regular inputs holding 5000 supersegments: 24 B each, 4 B count per pixel and input,
    # output N slots of 24 B per pixel plus count and gamma
    assert bench.composite_bytes([reg] * 3, N, P, 5000) == 24 * 5000 + 4 * 3 * P + 24 * N * P + 8 * P
    # a compact input adds its offsets
    assert bench.composite_bytes([reg, cmp_], N, P, 10) == 24 * 10 + 4 * 2 * P + 4 * P + 24 * N * P + 8 * P


def _summary(tmp_path, digest, kernels):
    p = tmp_path / "pmc.md"
    p.write_text("# counters\n\npmc: " + json.dumps({"source_sha256": digest, "fetch_scale": 2.0,
                                                    "write_scale": 1.0, "kernels": kernels}) + "\n")
    return str(p)


def test_measured_traffic_reads_matching_summary(tmp_path, monkeypatch):
    k = {"composite_cat_kernel": {"fetch_kib": 100.0, "write_kib": 50.0, "dispatches": 3}}
    monkeypatch.setattr(bench, "PMC_SUMMARY", _summary(tmp_path, bench.source_digest(), k))
    b, why = bench.measured_traffic("composite_cat_kernel")
    assert why == "measured" and b == pytest.approx((100.0 * 2.0 + 50.0) * 1024.0)
    b, why = bench.measured_traffic("gen_kernel")
    assert b is None and "no counters" in why


def test_measured_traffic_refuses_other_sources(tmp_path, monkeypatch):
    k = {"composite_cat_kernel": {"fetch_kib": 1.0, "write_kib": 1.0, "dispatches": 1}}
    monkeypatch.setattr(bench, "PMC_SUMMARY", _summary(tmp_path, "0" * 64, k))
    b, why = bench.measured_traffic("composite_cat_kernel")
    assert b is None and "changed" in why
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("composite_cat_kernel")[0] is None
