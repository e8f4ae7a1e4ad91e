"""The rocprofv3 summary tool on small synthetic CSV files (CPU only)."""
import csv
import json

from paper_2502_11017_amd import profsum


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_stats_table_and_match(tmp_path):
    p = tmp_path / "s.csv"
    _write(p, ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [["void cur::k_pass<double, 64>(...)", 10, 5000000, 500000],
            ["cur::k_ctl(...)", 5, 1000000, 200000],
            ["rocblas_gemm", 2, 4000000, 2000000]])
    out = profsum.kernel_stats(str(p), match="cur::")
    assert "k_pass" in out and "k_ctl" in out and "rocblas" not in out.split("other kernels")[0]
    assert "other kernels" in out
    assert "50.0%" in out  # k_pass: 5 of 10 ms


def test_traffic_calibrated_by_the_copy_and_last_dispatches(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Value"]
    # FETCH_SIZE reads half of the true bytes (as on the part), WRITE_SIZE all of them
    copy = 1 << 20
    f_rows = [[1, "copyBuffer", copy / 1024 / 2]]
    w_rows = [[1, "copyBuffer", copy / 1024]]
    for d, kib in ((2, 100.0), (3, 200.0), (4, 300.0)):
        f_rows += [[d, "k_pass<double, 64>", kib / 2 / 2], [d, "k_pass<double, 64>", kib / 2 / 2]]  # two instances
        w_rows += [[d, "k_pass<double, 64>", kib]]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, hdr, f_rows)
    _write(wp, hdr, w_rows)
    rec = profsum.pass_traffic(str(fp), str(wp), "k_pass", copy)
    assert rec["launches"] == 3
    assert abs(rec["calibration"]["fetch_scale"] - 2.0) < 1e-12
    assert abs(rec["fetch_bytes_per_launch"] - 200.0 * 1024) < 1e-6
    assert abs(rec["write_bytes_per_launch"] - 200.0 * 1024) < 1e-6
    last = profsum.pass_traffic(str(fp), str(wp), "k_pass", copy, last=1)
    assert last["launches"] == 1 and abs(last["bytes_per_launch"] - 2 * 300.0 * 1024) < 1e-6
    json.dumps(rec)
