"""Host-side pieces of bench.py that need no GPU: the one-GPU guard and the rule that a
committed counter record is reported only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

RECORD = os.path.join(ROOT, "profiles", "k_ilut_wave_upwind74_traffic.json")


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sources_hash_is_deterministic_and_covers_the_kernels():
    h = bench._sources_sha256()
    assert h == bench._sources_sha256() and len(h) == 64


@pytest.mark.skipif(not os.path.exists(RECORD), reason="no committed counter record")
def test_traffic_record_is_consistent():
    with open(RECORD) as f:
        rec = json.load(f)
    scaled = 1024.0 * (rec["fetch_scale"] * rec["fetch_KiB_per_dispatch"]
                       + rec["write_scale"] * rec["write_KiB_per_dispatch"])
    assert abs(scaled - rec["bytes_per_dispatch"]) <= 1e-6 * scaled + 1024
    assert rec["dispatches"] > 0 and rec["kernel"] == "k_ilut_wave<float>"


@pytest.mark.skipif(not os.path.exists(RECORD), reason="no committed counter record")
def test_traffic_is_reported_only_for_the_measured_sources_and_workload(monkeypatch):
    with open(RECORD) as f:
        rec = json.load(f)
    monkeypatch.setattr(bench, "_sources_sha256", lambda: rec["sources_sha256"])
    k = rec["kernel"]
    assert bench._traffic(k, "upwind74", 32, False) == rec["bytes_per_dispatch"]
    # another kernel, workload, group size or independent-set order: no figure
    assert bench._traffic("k_ilut_wave<double>", "upwind74", 32, False) is None
    assert bench._traffic(k, "grid40", 32, False) is None
    assert bench._traffic(k, "upwind74", 0, False) is None
    assert bench._traffic(k, "upwind74", 32, True) is None
    # sources changed since the counters were taken: no figure
    monkeypatch.setattr(bench, "_sources_sha256", lambda: "0" * 64)
    assert bench._traffic(k, "upwind74", 32, False) is None
