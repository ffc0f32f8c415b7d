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
    value = bench.measured_traffic()
    assert value is not None, "profiles/leja_kernel_traffic.txt predates the kernel sources: retake the counters"
    with open(bench.TRAFFIC_FILE) as fh:
        line = [x for x in fh if x.startswith("traffic_bytes_per_launch_dirichlet512:")][0]
    assert value == float(line.split(":")[1])
    # any change of the hashed sources makes the value unavailable
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES[:-1])
    assert bench.measured_traffic() is None
