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


def test_measured_traffic_reads_matching_summary(tmp_path):
    k = {"composite_cat_kernel": {"fetch_kib": 100.0, "write_kib": 50.0, "dispatches": 3}}
    path = _summary(tmp_path, bench.source_digest(bench.COMPOSITE_SOURCES), k)
    b, why = bench.measured_traffic("composite_cat_kernel", path)
    assert why == "measured" and b == pytest.approx((100.0 * 2.0 + 50.0) * 1024.0)
    b, why = bench.measured_traffic("gen_kernel", path)
    assert b is None and "no traffic counters" in why


def test_measured_traffic_refuses_other_sources(tmp_path):
    k = {"composite_cat_kernel": {"fetch_kib": 1.0, "write_kib": 1.0, "dispatches": 1}}
    path = _summary(tmp_path, "0" * 64, k)
    b, why = bench.measured_traffic("composite_cat_kernel", path)
    assert b is None and "changed" in why
    assert bench.measured_traffic("composite_cat_kernel", str(tmp_path / "missing.md"))[0] is None


def test_measured_valu_reads_generation_summary(tmp_path):
    k = {"gen_kernel<float, 0, false>": {"valu_insts": 1.5e9, "dispatches": 2}}
    path = _summary(tmp_path, bench.source_digest(bench.GENERATE_SOURCES), k)
    v, why = bench.measured_valu("gen_kernel<float, 0, false>", path)
    assert why == "measured" and v == pytest.approx(1.5e9)
    # a composite digest does not vouch for the generation kernel's sources
    path = _summary(tmp_path, bench.source_digest(bench.COMPOSITE_SOURCES), k)
    assert bench.measured_valu("gen_kernel<float, 0, false>", path)[0] is None


def test_valu_peak_from_unit_counts():
    # 256 CUs x 4 SIMDs x 32 fp32 lanes per cycle x 2.4 GHz; twice that is the 157.3 TFLOP/s (FMA = 2)
    assert bench.VALU_PEAK_TLANE == pytest.approx(78.6, rel=1e-3)
