"""The measurement script's contract that needs no GPU: several GPUs are
refused before any device work, and the counter-measured traffic is
reported only while the sweep source it was taken with is unchanged."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    table = {
        "fp32": {"source_hash": bench.sweep_source_hash(), "bytes_per_launch": 123},
        "fp16": {"source_hash": "0000000000000000", "bytes_per_launch": 456},
        "d3q19_256": {"source_hash": bench.sweep_source_hash(bench.D3_SOURCES), "bytes_per_launch": 789},
        "d3q19_256_mrt": {"source_hash": bench.sweep_source_hash(), "bytes_per_launch": 1},
    }
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(table))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(path))
    assert bench.measured_traffic("fp32") == 123
    assert bench.measured_traffic("fp16") is None              # taken with another source
    assert bench.measured_traffic("d3q19_256") == 789          # keyed by the D3Q19 source
    assert bench.measured_traffic("d3q19_256_mrt") is None     # the 2-D hash does not fit it
    assert bench.measured_traffic("unknown") is None


def test_committed_traffic_table_is_well_formed():
    d = json.load(open(os.path.join(ROOT, "profiles", "sweep_traffic_membrane4096.json")))
    for key, e in d.items():
        assert len(e["source_hash"]) == 16
        assert e["bytes_per_launch"] == round((e["fetch_kib_raw"] * e["fetch_scale"]
                                              + e["write_kib_raw"] * e["write_scale"]) * 1024)
        # counters within a few per cent of the algorithmic bytes
        assert 0.99 < e["bytes_per_launch"] / e["algorithmic_bytes_per_launch"] < 1.1
