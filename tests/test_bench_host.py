"""Host-side checks of bench.py that need no GPU: a request for more than one GPU exits with
a message (this build runs on one GPU), incompatible mode combinations are refused, and the
counter-measured traffic is reported only for the kernel and workload it was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_exits_with_message():
    for n in ("2", "8"):
        r = _run("--gpus", n)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_gp_with_focal_refused():
    r = _run("--gp", "--refine-focal")
    assert r.returncode == 2 and "global positioning" in r.stderr


def test_traffic_only_for_its_kernel_and_workload():
    assert bench.measured_traffic("schur_cam", "large") is None
    assert bench.measured_traffic("schur_point", "xl") is None
    v = bench.measured_traffic("schur_point", "large")
    assert v is None or v > 0.0   # None once the library sources differ from the measured ones
