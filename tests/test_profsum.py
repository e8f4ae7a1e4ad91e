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


def test_level_table_splits_selections_and_levels(tmp_path):
    """Two selections of two levels each on one stream; the first is skipped.
    Level 0 of the second: 0.010 ms wall starting at its panel copy, with
    pass 2 us, fresh 1 us, ctl 3 us; level 1: the merge set-up and one ctl."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for base in (0, 1_000_000):
        rows += [["void cur::k_amax<double>(...)", base, base + 1000],
                 ["void cur::k_panel_from_A<double>(...)", base + 2000, base + 3000],
                 ["void cur::k_fresh<double, 64>(...)", base + 4000, base + 5000],
                 ["void cur::k_pass<double, 64>(...)", base + 5000, base + 7000],
                 ["void cur::k_ctl<double, 64>(...)", base + 9000, base + 12000],
                 ["cur::k_merge_init(...)", base + 20000, base + 21000],
                 ["void cur::k_ctl<double, 64>(...)", base + 22000, base + 26000]]
    p = tmp_path / "t.csv"
    _write(p, hdr, rows)
    out = profsum.level_table(str(p), skip=1).splitlines()
    assert out[0].startswith("1 selection(s), 2 levels")
    lv0 = out[2].split()
    assert lv0[:7] == ["0", "0.010", "0.002", "0.001", "0.003", "0.001", "0.003"]
    lv1 = out[3].split()
    assert lv1[:7] == ["1", "0.006", "0.000", "0.000", "0.004", "0.001", "0.001"]
    assert out[4].split()[0] == "all"


def test_level_table_keeps_a_polish_panel_copy_in_its_level(tmp_path):
    """A polish level copies its panel after its merge set-up: one level, not two."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [["void cur::k_amax<double>(...)", 0, 1000],
            ["void cur::k_panel_from_A<double>(...)", 2000, 3000],
            ["void cur::k_ctl<double, 64>(...)", 4000, 5000],
            ["cur::k_merge_init(...)", 6000, 7000],
            ["void cur::k_panel_from_A<double>(...)", 7000, 9000],
            ["void cur::k_ctl<double, 64>(...)", 9000, 10000]]
    p = tmp_path / "t.csv"
    _write(p, hdr, rows)
    out = profsum.level_table(str(p)).splitlines()
    assert out[0].startswith("1 selection(s), 2 levels")
    lv1 = out[3].split()
    assert lv1[:2] == ["1", "0.004"] and lv1[7] == "3"


def test_mfma_table_flops_and_busy_share(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for d in (1, 2):
        # two shader-engine instances of each SQ counter; a 1 ms dispatch
        t0 = d * 10_000_000
        for ctr, v in (("SQ_INSTS_VALU_MFMA_MOPS_F64", 1e6), ("SQ_VALU_MFMA_BUSY_CYCLES", 1.2288e9 / 2)):
            rows += [[d, "k_resid_mfma<double>", ctr, v, t0, t0 + 1_000_000]] * 2
        rows += [[d, "k_resid_mfma<double>", "GRBM_GUI_ACTIVE", 7e6, t0, t0 + 1_000_000]]
    p = tmp_path / "c.csv"
    _write(p, hdr, rows)
    f = profsum.mfma_table(str(p), simds=1024, ghz=2.4).splitlines()[1].split()
    assert f[1] == "2" and f[2] == "1000.0" and f[3] == "1.024"  # 2e6 MOPS x 512 per dispatch
    assert f[-2] == "1.0"  # 1.024 GFLOP in 1 ms
    assert f[-1] == "0.500"  # 1.2288e9 busy cycles / (1e6 ns x 2.4 GHz x 1024 SIMDs)


def test_duration_percentiles(tmp_path):
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [["void cur::k_fresh<double, 64>(...)", 0, 1000 * (i + 1)] for i in range(11)]
    p = tmp_path / "t.csv"
    _write(p, hdr, rows)
    line = profsum.duration_table(str(p)).split()
    assert line[:3] == ["k_fresh", "11", "launches:"]
    assert line[4] == "2.0" and line[6] == "6.0" and line[8] == "10.0" and line[10] == "11.0"


def test_lds_table_bytes_rate_and_conflict_share(tmp_path):
    p = tmp_path / "l.csv"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for d in (1, 2):  # two dispatches of 1 ms each, counters split over two instances
        t0 = 10_000_000 * d
        for ctr, v in (("SQ_INSTS_LDS_LOAD_BANDWIDTH", 1e8), ("SQ_LDS_IDX_ACTIVE", 4e6), ("SQ_LDS_BANK_CONFLICT", 1e6)):
            rows += [[d, "k_resid_mp<1>", ctr, v / 2, t0, t0 + 1_000_000]] * 2
    _write(p, hdr, rows)
    f = profsum.lds_table(str(p), cus=256, ghz=2.4).splitlines()[1].split()
    # 1e8 x 64 B = 6.4 GB per dispatch in 1 ms: 6.4 TB/s of 78.6 (128 B x 256 CUs x 2.4 GHz)
    assert f[-5] == "1000.0" and f[-4] == "6.40" and f[-3] == "6.4"
    assert abs(float(f[-2]) - 6.4e3 / (128 * 256 * 2.4)) < 1e-3
    assert f[-1] == "0.250"


def test_waits_table_shares_of_wave_cycles(tmp_path):
    p = tmp_path / "w.csv"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for ctr, v in (("SQ_WAVE_CYCLES", 1000.0), ("SQ_WAIT_ANY", 400.0), ("SQ_WAIT_INST_ANY", 250.0),
                   ("SQ_ACTIVE_INST_ANY", 200.0), ("SQ_ACTIVE_INST_VALU", 100.0)):
        rows += [[1, "k_resid_mp<1>", ctr, v / 2, 0, 1000]] * 2  # two instances
    _write(p, hdr, rows)
    f = profsum.waits_table(str(p)).splitlines()[1].split()
    assert f[-7:-3] == ["0.400", "0.250", "0.200", "0.100"]
    assert f[-3] == "nan"  # a counter the run did not collect
