"""The bench's command line on a host without a GPU: the multi-GPU request is
refused before anything touches a device, and the traffic figure follows
the de/gridding source it was measured on."""

import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    t = bench.KWINDOW_TRAFFIC["convex"]
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    got = bench.measured_traffic("convex")
    assert (got is not None) == (sha == t["sha256_16"])
    # any other source text drops the figure
    other = tmp_path / "k.hip"
    other.write_text("// a different kernel\n")
    monkeypatch.setitem(bench.KWINDOW_TRAFFIC, "convex", dict(t, src=str(other)))
    assert bench.measured_traffic("convex") is None
    assert bench.measured_traffic("decentral") is None
