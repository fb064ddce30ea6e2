"""Host logic of the measurement tools (no GPU): the rocprofv3 counter summary that
turns FETCH_SIZE / WRITE_SIZE into bytes per launch, and bench.py's refusal of
more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_1907_01995_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COLS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(COLS)
        for i, (name, value) in enumerate(rows):
            w.writerow([i + 1, i + 1, name, counter, float(value)])


SWEEP = "void rac::(anonymous namespace)::k_sweep2<float, 4, 16>(rac::(anonymous namespace)::Sweep2Args)"
COPY = "__amd_rocclr_copyBuffer"


def test_traffic_scales_each_counter_by_the_calibration_copy(tmp_path):
    copy_bytes = 256 << 20
    # the counter reads half the bytes a copy fetches (scale 2) and all it writes (scale 1);
    # other copies of the run are left out of the calibration, also a workload's upload of
    # 60% of the calibration size (only copies within 10% of the largest count)
    fetch_rows = [(SWEEP, 1000.0), (SWEEP, 1200.0), (COPY, copy_bytes / 2048.0), (COPY, copy_bytes / 2048.0),
                  (COPY, 0.6 * copy_bytes / 2048.0), (COPY, 3.0)]
    write_rows = [(SWEEP, 300.0), (SWEEP, 500.0), (COPY, copy_bytes / 1024.0), (COPY, 0.6 * copy_bytes / 1024.0),
                  (COPY, 1.0)]
    fa, wa = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_counters(fa, "FETCH_SIZE", fetch_rows)
    write_counters(wa, "WRITE_SIZE", write_rows)
    out = tmp_path / "traffic.json"
    profsum.main(["traffic", "--fetch", str(fa), "--write", str(wa), "--kernel", "k_sweep2",
                  "--copy-bytes", str(copy_bytes), "--launch-bytes", "1000000", "--out", str(out)])
    rec = json.loads(out.read_text())
    assert rec["kernel"] == "k_sweep2<float, 4, 16>"
    assert rec["copy_dispatches"] == [2, 1]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    expect = 1100.0 * 1024 * 2.0 + 400.0 * 1024 * 1.0      # mean KiB per dispatch, scaled
    assert rec["traffic_bytes_per_launch"] == pytest.approx(expect)
    assert rec["traffic_over_algorithmic"] == pytest.approx(expect / 1e6)
    assert rec["source_sha256"] == profsum.source_hash("k_sweep2") and len(rec["source_sha256"]) == 64


def test_traffic_needs_the_calibration_copies(tmp_path):
    fa, wa = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_counters(fa, "FETCH_SIZE", [(SWEEP, 10.0)])
    write_counters(wa, "WRITE_SIZE", [(SWEEP, 10.0)])
    with pytest.raises(SystemExit):
        profsum.main(["traffic", "--fetch", str(fa), "--write", str(wa), "--kernel", "k_sweep2",
                      "--copy-bytes", "1024", "--out", str(tmp_path / "t.json")])


def test_short_kernel_names():
    assert profsum.short_name(SWEEP) == "k_sweep2<float, 4, 16>"
    assert profsum.short_name("void rac::k_zdual(long, int)") == "k_zdual"
    assert profsum.short_name(COPY) == COPY


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
