"""The bench's contract pieces that need no GPU: it refuses more than one
GPU, and its byte counts are the ones its roofline states."""
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


def test_algorithmic_bytes():
    # per update: the state read once and written once + one occupancy word
    # per cell written and read once (8 / rho per particle)
    assert bench.floor_bytes_per_update("fp32", 10) == pytest.approx(56.8)
    assert bench.floor_bytes_per_update("fp64", 5) == pytest.approx(97.6)
    # the roofline entry of one launch of the 10^7-particle fluid
    r = bench.roofline("fp32", 10_000_000, 1_000_000, 100.0, traffic=6.0e8)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(5.68e8)
    assert r["achieved"] == pytest.approx(5680.0)
    assert r["frac"] == pytest.approx(0.71)
    assert r["traffic_over_algorithmic"] == pytest.approx(6.0e8 / 5.68e8)
    # the layout's own figure: state and 4-byte tag read once and written once
    assert bench.layout_bytes_per_particle("fp32") == 64.0
    assert bench.layout_bytes_per_particle("fp64") == 104.0
    assert r["layout_GBs"] == pytest.approx(6400.0)


def test_measured_traffic_is_tied_to_the_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    from paper_1801_10187_amd.build import kernel_hash
    got = bench.measured_traffic("fp32")
    if rec.get("kernel_hash") == kernel_hash():
        assert got == rec["bytes_per_launch"]["srd_100c_rho10_mbthermo"]["fp32"]
        # the counters read close to the layout's bytes (no wasted re-reads)
        assert 1.0 < got / (64.0 * 1e7) < 1.1
    else:
        assert got is None
