"""Host-only checks of bench.py's contract (no GPU): more than one GPU is
refused with a message, and the HBM traffic figure is taken from the
committed counter summary only while that summary matches the kernel
source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    # the committed summary gives a positive byte count while it matches the
    # kernel source (None once the source has changed since the counters)
    t = bench.measured_traffic()
    assert t is None or t > 0
    # a different kernel source: the old counters no longer apply
    src = tmp_path / "sysblk.hip"
    src.write_bytes(open(bench.KERNEL_SRC, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.measured_traffic() is None
