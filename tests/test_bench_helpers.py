"""Host-side checks of the benchmark's bookkeeping: the rocprofv3 summaries
(counter scaling by the calibration copy, kernel-to-stage mapping, copies
left out), the byte models, the radix pass rule, and the refusal of runs on
more than one GPU.  No GPU is used."""

import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _counter_csv(path, counter, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


BWD = "void inpc::k_tile_bwd<float, 16, false, 8, 1>(inpc::GpuView const*, int)"
RED = "void inpc::k_point_reduce_q<16>(inpc::GpuView const*, int)"


def test_counter_summary_scales_by_the_calibration_copy(tmp_path):
    # the 1 GiB copy reads as 512 Ki KiB of FETCH_SIZE (scale 2) and 1 Gi B of WRITE_SIZE (scale 1)
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    n = bench.COUNTER_STEPS
    _counter_csv(f, "FETCH_SIZE", [(bench.RUNTIME_COPY, 524288.0)] + [(BWD, 1000.0)] * n + [(RED, 10.0)] * n)
    _counter_csv(w, "WRITE_SIZE", [(bench.RUNTIME_COPY, 1048576.0)] + [(BWD, 100.0)] * n + [(RED, 1.0)] * n)
    md, rec = bench.summarize_counters(str(f), str(w))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["per_launch_bytes"]["blend_bwd"] == pytest.approx((2 * 1000.0 + 100.0) * 1024)
    assert rec["per_launch_bytes"]["point_reduce"] == pytest.approx((2 * 10.0 + 1.0) * 1024)
    # whole step: every dispatch of the COUNTER_STEPS steps, divided by the step count
    assert rec["step_bytes"] == pytest.approx((2 * 1010.0 + 101.0) * 1024)
    assert bench.RUNTIME_COPY not in md and "k_point_reduce_q<16>" in md


def test_counter_summary_rejects_a_kernel_without_a_stage(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(bench.RUNTIME_COPY, 524288.0), ("void inpc::k_new_kernel(int)", 5.0)])
    _counter_csv(w, "WRITE_SIZE", [(bench.RUNTIME_COPY, 1048576.0), ("void inpc::k_new_kernel(int)", 5.0)])
    with pytest.raises(ValueError, match="k_new_kernel"):
        bench.summarize_counters(str(f), str(w))


def test_kernel_statistics_leave_out_runtime_copies(tmp_path):
    p = tmp_path / "s.csv"
    cols = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for name, calls, tot in [(bench.RUNTIME_COPY, 400, 9_000_000), (BWD, 4, 2_000_000), (RED, 4, 1_000_000)]:
            w.writerow({"Name": name, "Calls": calls, "TotalDurationNs": tot, "AverageNs": tot / calls,
                        "Percentage": 0, "MinNs": 0, "MaxNs": 0, "StdDev": 0})
    md = bench.summarize_stats(str(p), "title", "cmd")
    rows = [l for l in md.splitlines() if l.startswith("| `")]
    assert len(rows) == 2 and "k_tile_bwd" in rows[0]
    assert "| 500.0 | 2000.0 | 66.7 |" in rows[0] and "| 250.0 | 1000.0 | 33.3 |" in rows[1]


def test_per_splat_model_of_the_backward():
    # the per-splat byte model of the tile backward on the 8M-point 1080p step
    # (M, M_b, P measured), as recomputed independently of this code: 2.371 GB
    b = bench.per_splat_bytes(N=8_000_000, M=24_853_905, M_b=24_021_187, P=1920 * 1080, F=16, feat_bytes=4,
                              pixel_bits=21)
    assert b["blend_bwd"] == 2_370_873_676


def test_radix_pass_rule():
    # fewest passes of at most 9 bits, digits of at least 7 bits
    assert bench.sort_passes("auto digits", "depth", 27) == 3
    assert bench.sort_passes("auto digits", "pixel", 15) == 2
    assert bench.sort_passes("auto digits", "pixel", 28) == 4
    assert bench.sort_passes("auto digits", "pixel", 8) == 1
    assert bench.sort_passes("depth sort 8-bit, pixel sort 11-bit", "depth", 27) == 4
    assert bench.sort_passes("depth sort 8-bit, pixel sort 11-bit", "pixel", 21) == 2


def test_compulsory_bytes_count_each_array_once():
    N, Nv, M, Mb, P, F, E, T = 1000, 800, 3000, 2900, 5000, 16, 1100, 100
    c = bench.compulsory_bytes(N, Nv, M, Mb, P, F, 4, 3, 2, 128, E=E, n_tiles=T)
    # projection: xyz, opacity, record, depth key + value + anchor word, payload rows
    assert c["project"] == 12 * N + 4 * N + 16 * N + 12 * N + 128 * Nv
    # three depth passes carry key, value and anchor word; two tile passes key and value
    assert c["sort_downsweep"] == 3 * 24 * N + 2 * 16 * E
    assert c["emit"] == 12 * N + 8 * E


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
