"""Summaries of profiler output: kernel statistics and the calibrated
per-dispatch HBM traffic."""
import csv
import json

from paper_2511_09546_amd import prof_summary


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_stats_sums_matching_kernels(tmp_path):
    _write(tmp_path / "1_kernel_stats.csv",
           ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [["gemm_f32_lds_kernel<float, 144, 4, 1, false, false>", 4, 4000,
             1000], ["permute_kernel", 9, 900, 100]])
    r = prof_summary.stats(str(tmp_path), r"lds_kernel<\w+, 144")
    assert r == {"gemm_f32_lds_kernel<float, 144, 4, 1, false, false>":
                 (4, 4000)}


def test_traffic_scales_by_the_copy(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    for d, c in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        (tmp_path / d).mkdir()
        # two dispatches of the kernel, one of another
        _write(tmp_path / d / "1_counter_collection.csv", hdr,
               [[1, "wide", c, 100.0], [2, "wide", c, 300.0],
                [3, "other", c, 7.0]])
        (tmp_path / ("c" + d)).mkdir()
        # the copy of 2048 KiB reads 1024 KiB by the fetch counter
        _write(tmp_path / ("c" + d) / "1_counter_collection.csv", hdr,
               [[1, "__amd_rocclr_copyBuffer", c,
                 1024.0 if c == "FETCH_SIZE" else 2048.0]])
    src = tmp_path / "k.hip"
    src.write_text("kernel")
    out = tmp_path / "t.json"
    prof_summary.main(["traffic", "--fetch", str(tmp_path / "f"),
                       "--write", str(tmp_path / "w"),
                       "--calib-fetch", str(tmp_path / "cf"),
                       "--calib-write", str(tmp_path / "cw"),
                       "--copy-bytes", str(2048 * 1024), "--kernel", "wide",
                       "--source", str(src), "--out", str(out)])
    r = json.loads(out.read_text())
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    assert r["fetch_bytes_per_launch"] == 2.0 * 200.0 * 1024
    assert r["write_bytes_per_launch"] == 200.0 * 1024
    assert r["dispatches"] == 2 and len(r["gemm_source_sha256"]) == 64
