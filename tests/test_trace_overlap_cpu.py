"""The device-overlap summary of per-process kernel traces."""
import csv

from paper_2511_09546_amd import trace_overlap


def test_overlap_counts_processes_in_flight():
    per = {"a": [(0, 10), (20, 30)], "b": [(5, 25)], "c": [(40, 50)]}
    r = trace_overlap.overlap(per)
    # busy: [0, 30] and [40, 50]; two processes at once in [5, 10], [20, 25]
    assert r["device_busy_s"] * 1e9 == 40
    assert r["two_or_more_s"] * 1e9 == 10
    assert r["max_processes_in_flight"] == 2
    assert r["busy_s"]["a"] * 1e9 == 20 and r["busy_s"]["b"] * 1e9 == 20
    # touching kernels of two processes do not overlap
    r = trace_overlap.overlap({"a": [(0, 10)], "b": [(10, 20)]})
    assert r["two_or_more_s"] == 0 and r["max_processes_in_flight"] == 1


def test_reads_rocprof_csv(tmp_path, capsys):
    for pid, rows in (("11", [(0, 100)]), ("12", [(50, 150), (160, 170)])):
        with open(tmp_path / f"{pid}_kernel_trace.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Kind", "Kernel_Name", "Start_Timestamp",
                        "End_Timestamp"])
            for a, b in rows:
                w.writerow(["KERNEL_DISPATCH", "k", a, b])
    assert trace_overlap.main([str(tmp_path)]) == 0
    out = capsys.readouterr().out
    assert "2 processes with kernels" in out
    assert "largest number of processes in flight: 2" in out
