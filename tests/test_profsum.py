"""Host logic of the rocprofv3 summariser (synthetic CSV files; no GPU)."""

import csv
import os
import subprocess
import sys

from paper_2305_19013_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_classes():
    assert profsum.kernel_class("void ecg::(anonymous namespace)::k_update_mfma<double, 32, 16>(int)") == "cgs2_update"
    assert profsum.kernel_class("k_gram_mfma<double, 16, 16>") == "cgs2_gram"
    assert profsum.kernel_class("k_reduce_chunks_stage<double>") == "cgs2_gram_reduce"
    assert profsum.kernel_class("k_spmm_grid_lds<double, 32, 4>") == "spmm"
    assert profsum.kernel_class("k_small_mfma<double, double, 32, true>") == "final_update"
    assert profsum.kernel_class("k_small_mfma<double, double, 32, false>") == "times_small"
    assert profsum.kernel_class("k_small_gram_mfma<double, 32, true>") == "small_gram"
    assert profsum.kernel_class("something_else") == "other"


def test_summary_calibrates_counters(tmp_path):
    th = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    _write(str(tmp_path / "t" / "host" / "1_kernel_trace.csv"), th,
           [["__amd_rocclr_copyBuffer", 0, 100], ["k_update_mfma<double, 32, 16>", 0, 2000],
            ["k_update_mfma<double, 32, 16>", 0, 4000], ["k_gram_mfma<double, 32, 16>", 0, 1000]])
    ch = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy reads half of the 1 GiB per FETCH_SIZE (factor 2) and all of it per WRITE_SIZE
    _write(str(tmp_path / "f" / "host" / "1_counter_collection.csv"), ch,
           [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288], [2, "k_update_mfma<double, 32, 16>", "FETCH_SIZE", 1000],
            [3, "k_update_mfma<double, 32, 16>", "FETCH_SIZE", 3000]])
    _write(str(tmp_path / "w" / "host" / "1_counter_collection.csv"), ch,
           [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576], [2, "k_update_mfma<double, 32, 16>", "WRITE_SIZE", 10],
            [3, "k_update_mfma<double, 32, 16>", "WRITE_SIZE", 30]])
    out = subprocess.run([sys.executable, "-m", "paper_2305_19013_amd.profsum", "--trace", str(tmp_path / "t"),
                          "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w")], cwd=ROOT,
                         capture_output=True, text=True, check=True).stdout
    # update: mean of 2000 and 4000 ns; traffic per dispatch (2*2000 KiB*1024 + 40*1024) / 2
    assert "cgs2_update: rocprofv3 0 ms over 2 launches (mean 3.0 µs)" in out
    want = (2.0 * 4000 * 1024 + 40 * 1024) / 2
    assert f"traffic_bytes_per_launch cgs2_update {want:.6e}" in out
    assert "kernels_sha256_16 " in out
