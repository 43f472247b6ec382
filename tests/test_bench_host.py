"""Host-side logic of bench.py (no GPU): the one-GPU guard, the paired
per-layer deposit check, and the lookup of recorded HBM traffic, which must
refuse counters taken for other kernel sources, another workload or other
knobs."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_paired_layers_accepts_equal_and_rejects_a_shifted_layer():
    rng = np.random.default_rng(3)
    y = rng.gamma(4.0, 1.0, size=(400, 20)) * np.linspace(1, 3, 20)
    same = bench.paired_layers(y.copy(), y)
    assert same["pass_"] and same["worst_rel_big_layers"] == 0.0 and same["layers"] == 20
    noisy = bench.paired_layers(y + rng.normal(0, 1e-6, y.shape), y)
    assert noisy["pass_"]
    x = y.copy()
    x[:, 7] *= 1.02                      # a 2 % bias on one big layer
    bad = bench.paired_layers(x, y)
    assert not bad["pass_"] and bad["worst_rel_big_layers"] > 0.015


def test_measured_traffic_matches_source_workload_and_knobs(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    rec = {"source_sha1": bench.kernel_source_hash(), "workload": "c4x10000",
           "entries": [{"knobs": [256, 3, 4], "bytes_per_step": 50.0},
                       {"knobs": [256, 3, 2], "bytes_per_step": 80.0}]}
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(1000.0, "c4x10000", (256, 3, 4)) == 50000.0
    assert bench.measured_traffic(1000.0, "c4x10000", (256, 3, 2)) == 80000.0
    assert bench.measured_traffic(1000.0, "c4x10000", (128, 6, 4)) is None
    assert bench.measured_traffic(1000.0, "c4x1250", (256, 3, 4)) is None
    rec["source_sha1"] = "0" * 40
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(1000.0, "c4x10000", (256, 3, 4)) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(1000.0, "c4x10000", (256, 3, 4)) is None


def test_source_hash_covers_the_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 40 and h == bench.kernel_source_hash()


def test_host_cpus_and_ungated_comparison():
    c = bench.host_cpus()
    assert 1 <= c["threads"] <= 16 and c["threads"] <= c["available"]
    rng = np.random.default_rng(5)
    y = rng.gamma(4.0, 1.0, size=(200, 10))
    r = bench.paired_layers(y + rng.normal(0, 0.5, y.shape), y, gate=False)
    assert "pass_" not in r and r["three_sigma_rel_median_big_layers"] > 0 and r["events"] == 200


def test_shower_roofline_takes_the_tail_out():
    """Shower-phase bytes per second: all algorithmic bytes less 108 B per
    tail step, over the kernel time outside the tail."""
    import bench
    res = dict(kern_ms=[300.0, 200.0], tail_ms=[200.0, 100.0], alg_bytes=1.0e12 + 108.0 * 1.0e6, tail_steps=1.0e6)
    r = bench.shower_roofline(res)
    assert abs(r["achieved"] - 1.0e12 / 0.2 / 1e9) < 1e-6
    assert abs(r["frac"] - 1.0e12 / 0.2 / 8.0e12) < 1e-12
    assert abs(r["kernel_ms_per_transport"] - 100.0) < 1e-9
    assert bench.shower_roofline(dict(kern_ms=[1.0], tail_ms=[1.0], alg_bytes=1.0, tail_steps=0.0)) is None
