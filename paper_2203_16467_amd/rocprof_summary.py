"""Summarise a rocprofv3 kernel trace (CSV output) as a markdown table.

    python -m paper_2203_16467_amd.rocprof_summary <rocprofv3 output dir> [--range NAME]

Per kernel symbol: calls, total / average / min / max duration; and per role
of the solver tick (row-forward, column, row-inverse FFT kernels, controller),
summed over the kernel variants that fill that role (LDS or register FFTs).
With --range, only dispatches that start inside the roctx range NAME (pushed
by bench.py around its timed steps; needs --marker-trace) are counted, so the
figures cover exactly the region the benchmark's own timers cover.
Streams the CSV files (a trace of millions of dispatches is fine).
"""

import argparse
import csv
import glob
import os
import re
import sys

ROLES = (("rowfwd", re.compile(r"k_rowfwd")), ("col", re.compile(r"k_col")),
         ("rowinv", re.compile(r"k_rowinv")), ("ctrl", re.compile(r"k_ctrl")))


def _files(root, suffix):
    return sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))


def marker_ranges(root, name):
    """(start, end) timestamps of every roctx range whose message is name."""
    out = []
    for f in _files(root, "marker_api_trace.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if any(v == name for v in row.values()):
                    out.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"])))
    return out


def short_name(k):
    k = re.sub(r"\(.*$", "", k)
    return k.replace("void ", "").replace("spff::", "")


def summarise(root, rng=None):
    ranges = marker_ranges(root, rng) if rng else None
    if rng and not ranges:
        raise SystemExit(f"no roctx range named {rng!r} in {root}")
    stats = {}
    for f in _files(root, "kernel_trace.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                t0, t1 = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
                if ranges and not any(a <= t0 <= b for a, b in ranges):
                    continue
                k = short_name(row["Kernel_Name"])
                d = (t1 - t0) * 1e-3  # us
                s = stats.setdefault(k, [0, 0.0, float("inf"), 0.0])
                s[0] += 1
                s[1] += d
                s[2] = min(s[2], d)
                s[3] = max(s[3], d)
    return stats


def table(stats):
    lines = ["| Kernel | Calls | Total ms | Average us | Min us | Max us |", "|---|---|---|---|---|---|"]
    for k, (n, tot, lo, hi) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {k} | {n} | {tot * 1e-3:.1f} | {tot / n:.2f} | {lo:.2f} | {hi:.2f} |")
    lines += ["", "| Role | Calls | Total ms | Average us |", "|---|---|---|---|"]
    for role, pat in ROLES:
        n = sum(v[0] for k, v in stats.items() if pat.search(k))
        tot = sum(v[1] for k, v in stats.items() if pat.search(k))
        if n:
            lines.append(f"| {role} | {n} | {tot * 1e-3:.1f} | {tot / n:.2f} |")
    return "\n".join(lines)


def counters(root, kernel_regex=None):
    """Mean Counter_Value per dispatch, per (kernel symbol, counter), from a
    --pmc run's counter_collection.csv."""
    pat = re.compile(kernel_regex) if kernel_regex else None
    acc = {}
    for f in _files(root, "counter_collection.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                k = short_name(row["Kernel_Name"])
                if pat and not pat.search(k):
                    continue
                key = (k, row["Counter_Name"])
                a = acc.setdefault(key, [0, 0.0])
                a[0] += 1
                a[1] += float(row["Counter_Value"])
    return {key: (n, v / n) for key, (n, v) in acc.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("root")
    ap.add_argument("--range", default=None)
    ap.add_argument("--pmc", action="store_true", help="summarise a --pmc run (mean value per dispatch)")
    ap.add_argument("--kernel", default=None, help="regex on the kernel symbol (with --pmc)")
    a = ap.parse_args(argv)
    if a.pmc:
        for (k, c), (n, v) in sorted(counters(a.root, a.kernel).items()):
            print(f"{k} | {c} | dispatches {n} | mean per dispatch {v:.3f}")
    else:
        print(table(summarise(a.root, a.range)))


if __name__ == "__main__":
    main(sys.argv[1:])
