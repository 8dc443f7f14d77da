"""Device overlap of several processes from rocprofv3 kernel traces.

    python -m paper_2511_09546_amd.trace_overlap DIR

reads every ``*_kernel_trace.csv`` under DIR (rocprofv3 --kernel-trace
--output-format csv writes one per traced process, e.g. the worker
processes of the request loop) and prints a short text summary: per
process the kernels and the time some kernel of it was running; for the
whole device the time any kernel was running, the time kernels of two or
more processes were running at once, the time-weighted distribution of the
number of processes with a kernel in flight, and the largest such number.
Timestamps are the profiler's, common to all processes of the machine.
"""
from __future__ import annotations

import csv
import glob
import os
import sys


def _intervals(path):
    """[(start, end)] in ns of the kernel dispatches of one trace file."""
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            if b > a:
                out.append((a, b))
    return out


def _union(iv):
    """Total length of the union of intervals."""
    tot, cur_a, cur_b = 0, None, None
    for a, b in sorted(iv):
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                tot += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        tot += cur_b - cur_a
    return tot


def overlap(per_proc):
    """Summary of {process: [(start, end)]}: dict of the quantities in the
    module doc (times in seconds)."""
    ev = []
    for p, iv in per_proc.items():
        for a, b in iv:
            ev.append((a, 1, p))
            ev.append((b, -1, p))
    # ends before starts at equal times: touching kernels do not overlap
    ev.sort(key=lambda t: (t[0], t[1]))
    active = {}
    hist = {}
    last = None
    for t, s, p in ev:
        if last is not None and t > last:
            k = sum(1 for v in active.values() if v > 0)
            hist[k] = hist.get(k, 0) + (t - last)
        active[p] = active.get(p, 0) + s
        last = t
    busy = sum(v for k, v in hist.items() if k >= 1)
    multi = sum(v for k, v in hist.items() if k >= 2)
    return {
        "processes": len(per_proc),
        "kernels": {p: len(iv) for p, iv in per_proc.items()},
        "busy_s": {p: _union(iv) / 1e9 for p, iv in per_proc.items()},
        "device_busy_s": busy / 1e9,
        "two_or_more_s": multi / 1e9,
        "processes_in_flight_s": {k: v / 1e9 for k, v in sorted(hist.items())
                                  if k >= 1},
        "max_processes_in_flight": max([k for k, v in hist.items() if v > 0],
                                       default=0),
    }


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if len(argv) != 1:
        print(__doc__, file=sys.stderr)
        return 2
    files = sorted(glob.glob(os.path.join(argv[0], "**", "*_kernel_trace.csv"),
                             recursive=True))
    per = {}
    for f in files:
        iv = _intervals(f)
        if iv:
            per[os.path.basename(f).split("_")[0]] = iv
    r = overlap(per)
    print(f"traces: {len(files)} files, {r['processes']} processes with "
          "kernels")
    for p in sorted(per):
        print(f"  process {p}: {r['kernels'][p]} kernels, busy "
              f"{r['busy_s'][p]:.3f} s")
    print(f"device busy (any kernel running): {r['device_busy_s']:.3f} s")
    print(f"kernels of >= 2 processes running at once: "
          f"{r['two_or_more_s']:.3f} s "
          f"({r['two_or_more_s'] / max(r['device_busy_s'], 1e-30):.1%} of "
          "the busy time)")
    print("time with k processes in flight: " + ", ".join(
        f"{k}: {v:.3f} s" for k, v in r["processes_in_flight_s"].items()))
    print(f"largest number of processes in flight: "
          f"{r['max_processes_in_flight']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
