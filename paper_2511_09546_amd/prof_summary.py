"""Summaries of rocprofv3 output for the roofline record.

    python -m paper_2511_09546_amd.prof_summary stats DIR REGEX
        kernels whose name matches REGEX in the --stats files under DIR:
        calls, total and average duration (one line per kernel and the sum)

    python -m paper_2511_09546_amd.prof_summary traffic --fetch DIR
        --write DIR --calib-fetch DIR --calib-write DIR --copy-bytes N
        --kernel REGEX [--source FILE] [--workload TEXT] [--out JSON]
        HBM bytes per dispatch of the kernels matching REGEX from two
        counter passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
        scaled by what the same counter reads for a plain device copy of N
        bytes (the dispatches named *copyBuffer* in the calibration passes):
        scale = N / (1024 * mean reading).  Prints the record (JSON) and
        writes it to --out; --source adds the SHA-256 of that file, so a
        reader can tell whether the kernel changed since.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys


def _files(root, suffix):
    return sorted(glob.glob(os.path.join(root, "**", "*" + suffix),
                            recursive=True))


def stats(root, regex):
    """{kernel: (calls, total ns)} of the matching kernels."""
    pat = re.compile(regex)
    out = {}
    for f in _files(root, "_kernel_stats.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if pat.search(row["Name"]):
                    c, t = out.get(row["Name"], (0, 0))
                    out[row["Name"]] = (c + int(row["Calls"]),
                                        t + int(row["TotalDurationNs"]))
    return out


def counter_means(root, counter, regex):
    """(dispatches, mean value) of `counter` over the matching dispatches."""
    pat = re.compile(regex)
    vals = {}
    for f in _files(root, "_counter_collection.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                if not pat.search(row["Kernel_Name"]):
                    continue
                key = (f, row["Dispatch_Id"])
                vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} records for /{regex}/ under {root}")
    return len(vals), sum(vals.values()) / len(vals)


def traffic(a):
    nc_f, calib_f = counter_means(a.calib_fetch, "FETCH_SIZE", "copyBuffer")
    nc_w, calib_w = counter_means(a.calib_write, "WRITE_SIZE", "copyBuffer")
    sf = a.copy_bytes / (1024.0 * calib_f)
    sw = a.copy_bytes / (1024.0 * calib_w)
    n_f, fetch = counter_means(a.fetch, "FETCH_SIZE", a.kernel)
    n_w, write = counter_means(a.write, "WRITE_SIZE", a.kernel)
    rec = {"kernel": a.kernel, "workload": a.workload,
           "traffic_bytes_per_launch": 1024.0 * (fetch * sf + write * sw),
           "fetch_bytes_per_launch": 1024.0 * fetch * sf,
           "write_bytes_per_launch": 1024.0 * write * sw,
           "fetch_scale": sf, "write_scale": sw,
           "dispatches": min(n_f, n_w),
           "calibration": {"copy_bytes": a.copy_bytes,
                           "fetch_kib": calib_f, "write_kib": calib_w,
                           "dispatches": min(nc_f, nc_w)}}
    if a.source:
        with open(a.source, "rb") as fh:
            rec["gemm_source_sha256"] = hashlib.sha256(fh.read()).hexdigest()
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawTextHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("regex")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--source")
    t.add_argument("--workload", default="")
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        r = stats(a.dir, a.regex)
        calls = sum(c for c, _ in r.values())
        tot = sum(t for _, t in r.values())
        for name, (c, tt) in sorted(r.items(), key=lambda kv: -kv[1][1]):
            print(f"{c:8d} calls {tt / 1e6:10.1f} ms {tt / c / 1e3:9.2f} us  "
                  f"{name[:150]}")
        print(f"{calls:8d} calls {tot / 1e6:10.1f} ms "
              f"{tot / max(calls, 1) / 1e3:9.2f} us  (all matching)")
        return 0
    rec = traffic(a)
    txt = json.dumps(rec, indent=1)
    print(txt)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(txt + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
