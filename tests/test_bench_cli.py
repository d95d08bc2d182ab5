"""Host-side checks of the benchmark's command line and its traffic record
(no GPU: these paths exit or return before any device work)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_window_outside_the_ramp_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--start", "195", "--steps", "10"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "ramp" in r.stderr


def test_traffic_record_matches_the_kernel_sources():
    """The committed PMC record belongs to the kernel sources in the tree, so
    the benchmark reports the measured traffic rather than null."""
    sys.path.insert(0, ROOT)
    import bench
    for role in ("rowfwd", "rowinv"):
        t = bench.measured_traffic(role)
        assert t is not None and 15e6 < t < 25e6
