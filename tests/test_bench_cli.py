"""Host-side checks of the benchmark's command line and its traffic record
(no GPU: these paths exit or return before any device work)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_window_outside_the_ramp_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--start", "195", "--steps", "10"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "ramp" in r.stderr


def _record(path, sha, window):
    with open(path, "w") as f:
        f.write("# test record\n")
        f.write(f"kernel_source_sha256: {sha}\nwindow: {window}\n")
        f.write("rowfwd.read_kib_per_dispatch: 200.0\nrowfwd.write_kib_per_dispatch: 50.0\n")


def test_traffic_is_reported_only_for_the_measured_sources_and_window(tmp_path, monkeypatch):
    """roofline.traffic comes from a committed rocprofv3 --pmc record and is
    null unless that record was taken on the kernel sources being run and on
    the timed window being reported."""
    import bench
    rec = tmp_path / "pmc.txt"
    monkeypatch.setattr(bench, "PMC_RECORD", str(rec))
    assert bench.measured_traffic("rowfwd", "82..101") is None  # no record
    _record(rec, bench.kernel_source_hash(), "82..101")
    assert bench.measured_traffic("rowfwd", "82..101") == (200.0 + 50.0) * 1024.0
    assert bench.measured_traffic("rowfwd", "88..107") is None  # another window
    assert bench.measured_traffic("col", "82..101") is None     # another kernel
    _record(rec, "0" * 64, "82..101")
    assert bench.measured_traffic("rowfwd", "82..101") is None  # other sources


def test_committed_traffic_record_if_any_matches_the_sources():
    import bench
    if not os.path.exists(bench.PMC_RECORD):
        return
    text = open(bench.PMC_RECORD).read()
    assert f"kernel_source_sha256: {bench.kernel_source_hash()}" in text
