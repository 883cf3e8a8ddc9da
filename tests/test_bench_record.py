"""bench.py --record-traffic: the per-launch HBM bytes it derives from rocprofv3
counter CSVs, checked on small synthetic CSVs (no GPU)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

S3 = "void esbgk::stage_kernel<float, float, 32, 64, 4, 2, 1, false, 1, true>(esbgk::StageArgs)"
S2 = "void esbgk::stage_kernel<float, float, 32, 64, 4, 1, 0, false, 1, false>(esbgk::StageArgs)"
FI = "void esbgk::stage_kernel<float, float, 32, 64, 4, 1, 0, true, 1, false>(esbgk::StageArgs)"
COPY = "__amd_rocclr_copyBuffer"


def test_stage_class():
    assert bench.stage_class(S3) == "stage3"
    assert bench.stage_class(S2) == "stage2"
    assert bench.stage_class(FI) == "final"
    assert bench.stage_class("void esbgk::fill_maxwellian_kernel<float, 32, 64, 4>(esbgk::FillArgs<float>)") is None


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(rows):
            w.writerow([i + 1, name, counter, v])


def test_record_traffic_scales_by_the_copy_and_keeps_timed_dispatches(tmp_path):
    # a 1 MiB copy counted as 512 KiB fetched (x2) and 1024 KiB written (x1);
    # 2 warm-up and 3 timed dispatches per stage kernel
    seq = [(COPY, None)] + [(k, None) for _ in range(5) for k in (S2, S3, FI)]
    fetch = [(n, 512.0 if n == COPY else (100.0 if i <= 6 else 1000.0)) for i, (n, _) in enumerate(seq)]
    write = [(n, 1024.0 if n == COPY else (10.0 if i <= 6 else 300.0)) for i, (n, _) in enumerate(seq)]
    _write_counters(tmp_path / "fetch.csv", "FETCH_SIZE", fetch)
    _write_counters(tmp_path / "write.csv", "WRITE_SIZE", write)
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        for n in (S3, S2, FI):
            w.writerow([n, 5, 500000, 100000, 30.0, 50000, 150000, 1.0])
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for i, (n, _) in enumerate(seq):
            w.writerow([i + 1, n, 1000 * i, 1000 * i + (50000 if i <= 6 else 150000)])
    out = tmp_path / "traffic.json"
    env = dict(os.environ)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--record-traffic", str(tmp_path / "run_kernel_stats.csv"),
           str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"), "--calibrate-copy", "1", "--steps", "3",
           "--precision", "bf16"]  # bf16: the summary only, profiles/traffic.json is left alone
    text = subprocess.check_output(cmd, text=True, env=env, cwd=ROOT)
    assert "FETCH_SIZE x 2.000, WRITE_SIZE x 1.000" in text
    # timed dispatches only: 1000 KiB x 2 fetched, 300 KiB written, 150 us each
    for cls in ("stage2", "stage3", "final"):
        line = [l for l in text.splitlines() if l.startswith(f"| {cls} |")][0]
        cells = [c.strip() for c in line.strip("|").split("|")]
        assert cells[1] == "150.0"
        assert abs(float(cells[2]) - 1000 * 1024 * 2 / 1e6) < 0.05
        assert abs(float(cells[3]) - 300 * 1024 / 1e6) < 0.05
    assert not out.exists()
