"""bench.py --summarize-profile on small hand-made rocprofv3 CSV files: the
counter scale comes from the BitwiseOrFunctor copy alone (other elementwise
kernels do not enter it), kernel names lose namespaces, template arguments
and parameters, and the traffic per launch is the scaled mean."""
import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summary_scales_by_the_bitwise_or_copy(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.short_kernel_name(
        "void morph::(anonymous namespace)::col_and_kernel<false>(morph::(anonymous namespace)::RowsIn, int)") \
        == "col_and_kernel"
    assert bench.short_kernel_name("morph::(anonymous namespace)::pack_rows_kernel(int const*, int)") \
        == "pack_rows_kernel"
    assert bench.short_kernel_name("void rect_kernel<512>(morph::RectPage, int)") == "rect_kernel"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    cal = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<long, long, long, " \
          "at::native::BitwiseOrFunctor<long> >, std::array<char*, 2ul> >(int, ...)"
    other = "void at::native::vectorized_elementwise_kernel<4, at::native::BinaryFunctor<int, int, bool> >(int)"
    rect = "void morph::(anonymous namespace)::rect_kernel<512>(morph::RectPage, int)"
    # the copy moves 1 MiB each way; FETCH reads half of it, WRITE all of it
    fetch = [[1, cal, "FETCH_SIZE", 512], [2, other, "FETCH_SIZE", 99999], [3, rect, "FETCH_SIZE", 256],
             [4, rect, "FETCH_SIZE", 768]]
    write = [[1, cal, "WRITE_SIZE", 1024], [2, other, "WRITE_SIZE", 5], [3, rect, "WRITE_SIZE", 2048],
             [4, rect, "WRITE_SIZE", 0]]
    _write(str(tmp_path / "f" / "p_counter_collection.csv"), hdr, fetch)
    _write(str(tmp_path / "w" / "p_counter_collection.csv"), hdr, write)
    _write(str(tmp_path / "t" / "x_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [[rect, 2, 4000, 2000], [cal, 1, 1000, 1000]])
    out = tmp_path / "sum.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-profile",
                        "--trace-dir", str(tmp_path / "t"), "--fetch-dir", str(tmp_path / "f"),
                        "--write-dir", str(tmp_path / "w"), "--calib-bytes", str(1 << 20), "--out", str(out)],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    text = out.read_text()
    assert "FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000" in text
    line = [l for l in text.splitlines() if l.startswith("traffic rect_kernel ")][0]
    # mean FETCH 512 KiB x 2 + mean WRITE 1024 KiB x 1 = 2 MiB per launch
    assert "bytes_per_launch=%d " % (2 << 20) in line
    assert "| rect_kernel | 2 | 1.0 | 1.0 |" in text


def test_sq_summary_per_kernel_and_index(tmp_path):
    """bench.py --summarize-sq: counters summed per library kernel and divided
    by its waves, durations from the kernel trace of the same command, the
    VALU index against 256 CUs at 2.4 GHz; torch's helpers are left out."""
    col = "void morph::(anonymous namespace)::col_and_kernel<false>(morph::(anonymous namespace)::RowsIn, int)"
    other = "void at::native::vectorized_elementwise_kernel<4, at::native::BinaryFunctor<int, int, bool> >(int)"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # two dispatches of 1000 waves; 614 400 VALU each = 1 us at one per CU-cycle
    pmc = [[1, col, "SQ_WAVES", 1000], [1, col, "SQ_INSTS_VALU", 614400], [1, col, "SQ_INSTS_LDS", 3000],
           [2, col, "SQ_WAVES", 1000], [2, col, "SQ_INSTS_VALU", 614400], [2, col, "SQ_INSTS_LDS", 1000],
           [3, other, "SQ_WAVES", 50], [3, other, "SQ_INSTS_VALU", 7]]
    _write(str(tmp_path / "p" / "p_counter_collection.csv"), hdr, pmc)
    _write(str(tmp_path / "t" / "t_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [[col, 0, 2000], [col, 5000, 7000], [other, 8000, 9000]])
    out = tmp_path / "sq.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-sq",
                        "--sq-dir", str(tmp_path / "p"), "--trace-dir", str(tmp_path / "t"), "--out", str(out)],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    rows = [l for l in out.read_text().splitlines() if l.startswith("| ")]
    assert rows[0] == "| kernel | dispatches | waves / dispatch | LDS / wave | VALU / wave | average us | VALU / CU-cycle |"
    # LDS (3000 + 1000) / 2000 waves; VALU 614.4 per wave; 2 us each: index 0.50
    assert rows[1] == "| col_and_kernel<false> | 2 | 1000 | 2.0 | 614.4 | 2.0 | 0.50 |"
    assert not any("vectorized_elementwise" in l for l in rows)
