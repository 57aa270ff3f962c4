"""Host logic of the profiling summaries: the kernel-code hash ignores
comments, the counter summary scales by the copy calibration, and the trace
table groups launches by kernel and grid."""
import csv
import os

from paper_1611_02445_amd import profiling as P


def test_code_only_ignores_comments_and_spacing():
    a = "int f(int x) { // add one\n  return x + 1; /* done\n */ }\n"
    b = "int f(int x) {\n\treturn x + 1;   }"
    assert P._code_only(a) == P._code_only(b)
    assert P._code_only("a + b") != P._code_only("a - b")


def test_kernel_source_hash_is_stable():
    assert P.kernel_source_hash() == P.kernel_source_hash()
    assert len(P.kernel_source_hash()) == 16


def _write_csv(path, rows, fields):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counters_summary_scales_by_copy(tmp_path):
    f = ["Counter_Name", "Kernel_Name", "Grid_Size", "Counter_Value"]
    _write_csv(str(tmp_path / "f" / "x_counter_collection.csv"),
               [dict(Counter_Name="FETCH_SIZE", Kernel_Name="k_step<0>", Grid_Size=64, Counter_Value=100.0),
                dict(Counter_Name="FETCH_SIZE", Kernel_Name="k_step<0>", Grid_Size=64, Counter_Value=300.0),
                dict(Counter_Name="FETCH_SIZE", Kernel_Name="k_step<0>", Grid_Size=128, Counter_Value=999.0)], f)
    _write_csv(str(tmp_path / "w" / "x_counter_collection.csv"),
               [dict(Counter_Name="WRITE_SIZE", Kernel_Name="k_step<0>", Grid_Size=64, Counter_Value=50.0)], f)
    _write_csv(str(tmp_path / "cf" / "x_counter_collection.csv"),
               [dict(Counter_Name="FETCH_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=512.0)], f)
    _write_csv(str(tmp_path / "cw" / "x_counter_collection.csv"),
               [dict(Counter_Name="WRITE_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=1024.0)], f)
    d = P.counters_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                           1024.0 * 1024, "k_step<0>", "cmd", grid=64)
    # the copy moved 1 MiB each way; FETCH_SIZE read back 512 KiB (scale 2), WRITE_SIZE 1024 KiB (scale 1)
    assert d["copy_calibration"]["fetch_scale"] == 2.0 and d["copy_calibration"]["write_scale"] == 1.0
    assert d["hbm_read_bytes_per_launch"] == 200.0 * 1024 * 2
    assert d["hbm_write_bytes_per_launch"] == 50.0 * 1024
    assert d["dispatches"] == [2, 1]


def test_trace_table_groups_by_kernel_and_grid(tmp_path):
    f = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"]
    rows = [dict(Kernel_Name="k", Grid_Size_X=64, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=0, End_Timestamp=2000),
            dict(Kernel_Name="k", Grid_Size_X=64, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=0, End_Timestamp=4000),
            dict(Kernel_Name="k", Grid_Size_X=32, Grid_Size_Y=1, Grid_Size_Z=1, Start_Timestamp=0, End_Timestamp=1000)]
    _write_csv(str(tmp_path / "t" / "t_kernel_trace.csv"), rows, f)
    t = P.trace_table(str(tmp_path / "t"))
    assert t[("k", 64)] == (2, 3.0, 2.0, 4.0)
    assert t[("k", 32)] == (1, 1.0, 1.0, 1.0)


def test_counters_table_rows_and_calibrated_bytes(tmp_path):
    f = ["Counter_Name", "Kernel_Name", "Grid_Size", "Counter_Value"]
    _write_csv(str(tmp_path / "f" / "x_counter_collection.csv"),
               [dict(Counter_Name="FETCH_SIZE", Kernel_Name="k_calib_layout<double, 0, u>", Grid_Size=64,
                     Counter_Value=1000.0),
                dict(Counter_Name="FETCH_SIZE", Kernel_Name="k_calib_layout<double, 2, u>", Grid_Size=64,
                     Counter_Value=3000.0)], f)
    _write_csv(str(tmp_path / "i" / "x_counter_collection.csv"),
               [dict(Counter_Name="SQ_WAVES", Kernel_Name="k_calib_layout<double, 0, u>", Grid_Size=64,
                     Counter_Value=7.0)], f)
    _write_csv(str(tmp_path / "cf" / "x_counter_collection.csv"),
               [dict(Counter_Name="FETCH_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=512.0)], f)
    _write_csv(str(tmp_path / "cw" / "x_counter_collection.csv"),
               [dict(Counter_Name="WRITE_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=1024.0)], f)
    txt = P.counters_table([str(tmp_path / "f"), str(tmp_path / "i")],
                           [("xyz", "k_calib_layout<double, 0,", 64), ("zig", "k_calib_layout<double, 2,", None)],
                           "cmd", str(tmp_path / "cf"), str(tmp_path / "cw"), 1024.0 * 1024)
    lines = txt.splitlines()
    assert lines[0].endswith("cmd")
    xyz = [ln for ln in lines if ln.startswith("xyz")][0].split()
    zig = [ln for ln in lines if ln.startswith("zig")][0].split()
    # HBM read MB = 1000 KiB x 1024 x 2 (fetch scale) / 1e6; no WRITE_SIZE run
    # and no request-size counters: "-"
    assert xyz[1:] == ["2.0", "-", "-", "1000.0", "7.0"]
    assert zig[1:] == ["6.1", "-", "-", "3000.0", "-"]


def test_counters_table_bytes_by_request_size(tmp_path):
    f = ["Counter_Name", "Kernel_Name", "Grid_Size", "Counter_Value"]
    rows = [dict(Counter_Name=f"TCC_EA0_RDREQ_{b}B_sum", Kernel_Name="k", Grid_Size=1, Counter_Value=v)
            for b, v in ((32, 1000.0), (64, 2000.0), (128, 3000.0))]
    _write_csv(str(tmp_path / "r" / "x_counter_collection.csv"), rows, f)
    _write_csv(str(tmp_path / "cf" / "x_counter_collection.csv"),
               [dict(Counter_Name="FETCH_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=512.0)], f)
    _write_csv(str(tmp_path / "cw" / "x_counter_collection.csv"),
               [dict(Counter_Name="WRITE_SIZE", Kernel_Name="copyBuffer", Grid_Size=1, Counter_Value=1024.0)], f)
    txt = P.counters_table([str(tmp_path / "r")], [("k", "k", None)], "cmd", str(tmp_path / "cf"),
                           str(tmp_path / "cw"), 1024.0 * 1024)
    line = [ln for ln in txt.splitlines() if ln.startswith("k ")][0].split()
    # (32 * 1000 + 64 * 2000 + 128 * 3000) / 1e6 = 0.544 MB
    assert line[3] == "0.5"
