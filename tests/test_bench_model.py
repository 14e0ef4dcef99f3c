"""The benchmark's roofline arithmetic against the worked example the paper prints (Sect. 6:
the light-speed model of the 7-point smoother on a SuperMUC-NG node).  No GPU."""
import os

import bench

from test_oracle_pins import read_golden


def test_light_speed_model_reproduces_paper_numbers():
    g = read_golden("paper_light_speed.txt")
    node = bench.light_speed_glups(g["stream_gbs"][0], g["bytes_per_lup"][0])
    assert round(node, 2) == g["node_glups"][0]
    per_core_mlups = g["node_glups"][0] / g["cores"][0] * 1e3
    assert abs(per_core_mlups - g["core_mlups"][0]) < 1e-9
    assert g["measured_min_mlups"][0] / per_core_mlups >= g["min_fraction"][0]


def test_mi355x_smoother_light_speed():
    """24 B per update at 8 TB/s: 333 GLUP/s per sweep (what bench.py reports beside the
    measured GLUP/s)."""
    assert abs(bench.light_speed_glups(bench.HBM_PEAK_GBS, 24) - 333.33) < 0.01


def test_traffic_record_is_tied_to_kernel_source(tmp_path, monkeypatch):
    """A counter summary taken on other kernel source is not reported as traffic."""
    import json
    rec = {"source_sha256_16": "0" * 16, "n": 513, "bytes_per_launch": 1.0}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic(511 ** 3) is None
    rec["source_sha256_16"] = bench.source_hash(bench.SMOOTHER_SOURCE)
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(511 ** 3) == 1.0
    assert bench.measured_traffic(255 ** 3) is None


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
