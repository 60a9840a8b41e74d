"""bench.py's host-side contract (CPU): more than one GPU is refused with a message and exit
status 2 before anything touches a GPU; the workload table names every configuration the
legs read, with the sizes and step counts the measurement is quoted on."""

import os
import subprocess
import sys

from workloads import WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_table():
    for name in ("n64", "n512", "n2048", "n4096", "ensemble64", "long512", "orders512"):
        assert name in WORKLOADS, name
    assert WORKLOADS["n4096"]["N"] == 4096 and WORKLOADS["n2048"]["N"] == 2048
    assert WORKLOADS["ensemble64"]["nsim"] == 64
    assert WORKLOADS["long512"]["steps"] >= 10000
    assert all(WORKLOADS[k]["tol"] == 1e-12 for k in ("n512", "n2048", "n4096", "long512"))
