"""Host-side logic of bench.py, on the CPU: latency percentiles, the HBM
traffic figure that is only reported for the kernel sources it was measured
on, and the refusal of multi-GPU runs."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_percentile_interpolates_between_order_statistics():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert bench.percentile(xs, 0.0) == 1.0
    assert bench.percentile(xs, 1.0) == 5.0
    assert bench.percentile(xs, 0.5) == 3.0
    assert abs(bench.percentile(xs, 0.99) - 4.96) < 1e-12
    assert bench.percentile([], 0.5) is None


def _profile(tmp, sha, fetch="100", write="200"):
    os.makedirs(os.path.join(tmp, "profiles"))
    with open(os.path.join(tmp, "profiles", "fused_ply_65536_traffic.md"), "w") as f:
        f.write(f"- source_sha256: `{sha}`\n- fetch_bytes_per_launch: `{fetch}`\n"
                f"- write_bytes_per_launch: `{write}`\n")


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    tmp = str(tmp_path)
    csrc = os.path.join(tmp, "paper_2511_07312_amd", "csrc")
    os.makedirs(csrc)
    h = hashlib.sha256()
    for name, text in (("device.h", b"// device\n"), ("engine.hip", b"// engine\n")):
        with open(os.path.join(csrc, name), "wb") as f:
            f.write(text)
        h.update(text)
    _profile(tmp, h.hexdigest())
    monkeypatch.setattr(bench, "ROOT", tmp)
    assert bench.traffic_from_profile() == 300.0
    with open(os.path.join(csrc, "engine.hip"), "ab") as f:   # any edit invalidates it
        f.write(b"// changed\n")
    assert bench.traffic_from_profile() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_graph_split_times_exactly_the_requested_plies():
    for steps in (1, 5, 20, 63, 64, 65, 100, 6400, 6401):
        P, full, R = bench.graph_split(steps)
        assert P * full + R == steps
        assert 1 <= P <= bench.GRAPH_PLIES and 0 <= R < P
    assert bench.graph_split(20) == (20, 1, 0)
    assert bench.graph_split(6400) == (64, 100, 0)
