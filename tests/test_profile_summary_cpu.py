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
