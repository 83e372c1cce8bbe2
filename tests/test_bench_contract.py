"""Host-side checks of the benchmark script: the one-GPU guard, the counter
summaries it reads the HBM traffic from, and its oracle baseline leg.
Nothing here touches a GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2011_06856_amd.profile_summary import kernel_source_hash  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("name,units", [("stream_collide_f32_circular_1024", 1024 * 1024 * 256),
                                        ("push_step_f32_quadrant_2048", 2048 * 2048 * 1536)])
def test_committed_counter_summaries_are_self_consistent(name, units):
    """Algorithmic bytes = 8 B per FP32 site-velocity update (one read, one
    write) times the updates of one launch; traffic = the two counters scaled
    by the copy calibration, in bytes."""
    d = json.load(open(os.path.join(ROOT, "profiles", name + ".json")))
    assert d["launch_bytes"] == 8.0 * units
    traffic = (d["fetch_kib"] * d["fetch_factor"] + d["write_kib"] * d["write_factor"]) * 1024.0
    assert abs(traffic - d["traffic_bytes"]) <= 1e-9 * traffic
    # a launch writes the populations once; the push kernel also writes its
    # partial moment sums (24 FP32 values a site plus the tile-edge halo
    # parts), which the counters see as about 2% more at 1536 velocities
    w = d["write_kib"] * d["write_factor"] * 1024.0 / (4.0 * units)
    assert 0.995 < w < 1.03, w
    assert d["traffic_bytes"] >= 0.99 * d["launch_bytes"]
    md = open(os.path.join(ROOT, "profiles", name + ".md")).read()
    assert d["kernel_sha256"] in md and "rocprofv3" in md


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("k") is None
    rec = {"traffic_bytes": 123.0, "kernel_sha256": kernel_source_hash()}
    (tmp_path / "profiles" / "k.json").write_text(json.dumps(rec))
    assert bench.counter_traffic("k") == 123.0
    rec["kernel_sha256"] = "0" * 64
    (tmp_path / "profiles" / "k.json").write_text(json.dumps(rec))
    assert bench.counter_traffic("k") is None


def test_cpu_baseline_reports_the_oracle_on_a_bounded_sample():
    r = bench.cpu_baseline(0.0)
    assert r["kind"] == "oracle" and r["unit"] == "GSVUPS"
    assert r["value"] > 0 and r["cores"] >= 1
    assert "256x256" in r["sample"] and "1 steps" in r["sample"]
    one = r["single_core"]
    assert one["cores"] == 1 and one["value"] > 0
    assert r["cpu_model"]
    import oracle as O
    assert O.num_threads() == r["cores"]      # the thread count is restored
