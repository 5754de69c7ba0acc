"""Host-side logic of the benchmark (no GPU): the one-GPU refusal, the lookup
of the committed traffic figure, and the rocprofv3 summaries on small
synthetic databases with the columns rocprofv3 writes."""
import json
import os
import re
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2410_05865_amd import profiling  # noqa: E402

SMO = "void cc::(anonymous namespace)::k_smo1_z<double>(cc::StencilLevel, double, double const*, double const*, double*, int)"
COPY = "void cc::(anonymous namespace)::k_copy(long long, double const*, double*)"
LU = "void cc::(anonymous namespace)::k_lu_forward<8, double>(cc::LuDev, cc::LuTasks)"


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_lookup_checks_size_and_source(monkeypatch, tmp_path):
    f = tmp_path / "traffic.md"
    f.write_text("- grid: `256^3`\n- kernels.hip sha256[:16]: `0123456789abcdef`\n"
                 "- k_smo1_z<double>: FETCH_SIZE 1 KiB, WRITE_SIZE 1 KiB per dispatch (6 dispatches, grid 1048576 "
                 "work-items)\n- SMO-1 bytes per launch (calibrated): `5.0e+08`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "_src_hash", lambda: "0123456789abcdef")
    assert bench._traffic(256) == pytest.approx(5.0e8)
    assert bench._traffic(256, 1048576) == pytest.approx(5.0e8)   # the hook's schedule (16 planes)
    assert bench._traffic(256, 2097152) is None                    # another schedule (8 planes)
    assert bench._traffic(128) is None                     # another grid
    monkeypatch.setattr(bench, "_src_hash", lambda: "fedcba9876543210")
    assert bench._traffic(256) is None                     # the kernels changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench._traffic(256) is None


def _counter_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id int, kernel_name text, grid_size int, "
                "counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_summary_calibrates_with_the_copy_kernel(tmp_path):
    n = 64
    n3 = n ** 3
    true_kib = 8.0 * n3 / 1024.0
    # FETCH_SIZE reads half the true bytes, WRITE_SIZE all of them (as measured on the part)
    # build-time trials of other schedules first (dispatches 1-3), then the timing
    # hook: two back-to-back smoother launches, the copy kernel, the LU sweeps
    fe = [(1, SMO, 8 * n3 // 16, "FETCH_SIZE", 9.0), (2, SMO, 8 * n3 // 16, "FETCH_SIZE", 9.0),
          (3, LU, 100, "FETCH_SIZE", 3.0),
          (4, SMO, 4 * n3 // 16, "FETCH_SIZE", 1.5 * true_kib), (5, SMO, 4 * n3 // 16, "FETCH_SIZE", 1.5 * true_kib),
          (6, COPY, n3 // 4, "FETCH_SIZE", true_kib / 2), (7, LU, 100, "FETCH_SIZE", 10.0)]
    wr = [(1, SMO, 8 * n3 // 16, "WRITE_SIZE", 9.0), (2, SMO, 8 * n3 // 16, "WRITE_SIZE", 9.0),
          (3, LU, 100, "WRITE_SIZE", 1.0),
          (4, SMO, 4 * n3 // 16, "WRITE_SIZE", true_kib), (5, SMO, 4 * n3 // 16, "WRITE_SIZE", true_kib),
          (6, COPY, n3 // 4, "WRITE_SIZE", true_kib), (7, LU, 100, "WRITE_SIZE", 2.0)]
    _counter_db(tmp_path / "f.db", fe)
    _counter_db(tmp_path / "w.db", wr)
    text = profiling.traffic_summary(str(tmp_path / "f.db"), str(tmp_path / "w.db"), n, "abc")
    by = float(re.search(r"SMO-1 bytes per launch \(calibrated\): `([0-9.e+]+)`", text).group(1))
    # the hook's launches: 3 x 8 B per cell read after calibration, 8 B written
    assert by == pytest.approx(32.0 * n3)
    assert "(2 dispatches, grid" in text
    assert "measured/algorithmic = 1.280" in text
    assert "fetch x2.0000, write x1.0000" in text


def test_hook_run_is_split_from_trials_on_other_levels(tmp_path):
    """The build's last schedule trials (a coarser level: another grid) can
    directly precede the timing hook's launches of the same kernel."""
    n = 64
    n3 = n ** 3
    true_kib = 8.0 * n3 / 1024.0
    fe = [(1, SMO, n3 // 64, "FETCH_SIZE", 1.0), (2, SMO, n3 // 64, "FETCH_SIZE", 1.0),
          (3, SMO, n3 // 4, "FETCH_SIZE", 1.5 * true_kib), (4, SMO, n3 // 4, "FETCH_SIZE", 1.5 * true_kib),
          (5, COPY, n3 // 4, "FETCH_SIZE", true_kib / 2)]
    wr = [(1, SMO, n3 // 64, "WRITE_SIZE", 1.0), (2, SMO, n3 // 64, "WRITE_SIZE", 1.0),
          (3, SMO, n3 // 4, "WRITE_SIZE", true_kib), (4, SMO, n3 // 4, "WRITE_SIZE", true_kib),
          (5, COPY, n3 // 4, "WRITE_SIZE", true_kib)]
    _counter_db(tmp_path / "f.db", fe)
    _counter_db(tmp_path / "w.db", wr)
    text = profiling.traffic_summary(str(tmp_path / "f.db"), str(tmp_path / "w.db"), n, "abc")
    assert "(2 dispatches, grid" in text
    assert "measured/algorithmic = 1.280" in text


def test_kernel_stats_take_the_timing_hooks_dispatches(tmp_path):
    con = sqlite3.connect(tmp_path / "t.db")
    con.execute("create table kernels (name text, start int, end int, grid_x int, grid_y int, grid_z int)")
    # a trial (another schedule), a solve's launch between other kernels, then the hook's run of two
    rows = [(SMO, 0, 20_000, 32768, 4, 1), (LU, 30_000, 40_000, 1024, 1, 1),
            (SMO, 50_000, 60_000, 32768, 4, 1), (LU, 70_000, 80_000, 1024, 1, 1),
            (SMO, 100_000, 220_000, 262144, 4, 1), (SMO, 300_000, 426_000, 262144, 4, 1)]
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    text = profiling.kernel_stats_summary(str(tmp_path / "t.db"), n=256)
    assert "| k_smo1_z<double> | 4 | 0.28 |" in text
    assert "2 dispatches, average 123.0 us" in text


def test_counter_summary_averages_the_timing_hooks_launches(tmp_path):
    rows = [(1, SMO, 10, "TA_BUSY_avr", 99.0), (2, COPY, 500, "TA_BUSY_avr", 7.0),
            (3, SMO, 1000, "TA_BUSY_avr", 10.0), (4, SMO, 1000, "TA_BUSY_avr", 20.0),
            (5, COPY, 500, "TA_BUSY_avr", 5.0)]
    _counter_db(tmp_path / "c.db", rows)
    text = profiling.counters_summary(str(tmp_path / "c.db"))
    assert "k_smo1_z<double> (grid 1000 work-items, 2 dispatches): TA_BUSY_avr 15" in text
    assert "k_copy (grid 500 work-items, 1 dispatches): TA_BUSY_avr 5" in text


def test_lu_launch_summary_joins_bytes_and_durations(tmp_path):
    """Per launch of the timing hook's LU-correction: calibrated bytes from the
    counter runs and durations from the trace, the first correction left out."""
    n = 64
    n3 = n ** 3
    true_kib = 8.0 * n3 / 1024.0
    LB = "void cc::(anonymous namespace)::k_lu_backward<8, double, double>(cc::LuDev, cc::LuTasks)"
    # a trial launch, the copy kernel, then 3 corrections of (forward, forward, backward, backward)
    pat = [LU, LU, LB, LB]
    fe = [(1, LU, 100, "FETCH_SIZE", 50.0), (2, COPY, n3 // 4, "FETCH_SIZE", true_kib / 2)]
    wr = [(1, LU, 100, "WRITE_SIZE", 50.0), (2, COPY, n3 // 4, "WRITE_SIZE", true_kib)]
    did = 3
    for rep in range(3):
        for j, k in enumerate(pat):
            fe.append((did, k, 100, "FETCH_SIZE", 1000.0 * (j + 1) * (3 if rep == 0 else 1)))
            wr.append((did, k, 100, "WRITE_SIZE", 100.0))
            did += 1
    _counter_db(tmp_path / "f.db", fe)
    _counter_db(tmp_path / "w.db", wr)
    con = sqlite3.connect(tmp_path / "t.db")
    con.execute("create table kernels (name text, start int, end int, grid_x int, grid_y int, grid_z int)")
    rows, t = [], 0
    for rep in range(3):
        for j, k in enumerate(pat):
            d = (10_000 if j < 2 else 20_000) * (5 if rep == 0 else 1)
            rows.append((k, t, t + d, 64, 1, 1))
            t += d + 1000
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    text = profiling.lu_launch_summary(str(tmp_path / "f.db"), str(tmp_path / "w.db"), str(tmp_path / "t.db"), n)
    # launch 0: fetch 1000 KiB x 2 + write 100 KiB = 2100 KiB = 2.15 MB in 10 us
    assert "| 0 | k_lu_forward<8, double> | 10.0 | 2.2 | 215 |" in text
    assert "| 3 | k_lu_backward<8, double, double> | 20.0 | 8.3 | 415 |" in text
    assert "| all | 4 launches (3 corrections in the counter runs, 3 in the trace) | 60.0 |" in text
