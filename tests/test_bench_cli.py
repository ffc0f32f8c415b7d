"""bench.py's contract on the CPU: a request for several GPUs is refused with
a message, and the roofline traffic is read from the committed rocprofv3
summary only while the kernel sources still hash to the recorded value."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_read_only_for_current_sources(monkeypatch):
    """The counter summary's bytes are reported only while the kernel sources
    hash to the value recorded with them; a changed source set gives None."""
    kv = bench.traffic_record()
    if kv is not None and bench.sources_sha256() == kv.get("kernel_sources_sha256"):
        assert bench.measured_traffic() == float(kv[bench.TRAFFIC_KEY])
    else:
        assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES[:-1])
    assert bench.measured_traffic() is None
