"""Host logic of bench.py on the CPU: the counter and kernel-time summaries it writes under
profiles/, the source-hash guard on the recorded traffic, byte accounting, and the one-GPU rule."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

COLS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _pmc_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(COLS)
        for k, (name, v) in enumerate(rows):
            w.writerow([k + 1, k + 1, name, counter, v])


def test_pmc_summary_scales_by_the_copy_calibration(tmp_path):
    """A 1 GiB copy that reads FETCH_SIZE = 512 MiB and writes 1 GiB sets the scales 2 and 1;
    the bulk kernel's bytes per launch are its mean counters times those scales."""
    gib_kib = float(1 << 20)
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    G = bench.TRACKED["grid"]
    _pmc_csv(fetch, "FETCH_SIZE", [(bench.COPY_KERNEL, gib_kib / 2), (G, 1000.0),
                                   (G, 1002.0), ("other", 5.0)])
    _pmc_csv(write, "WRITE_SIZE", [(bench.COPY_KERNEL, gib_kib), (G, 3000.0),
                                   (G, 3000.0), ("other", 1.0)])
    out = tmp_path / "sum.txt"
    bench.pmc_summary(str(fetch), str(write), str(out), "cmd")
    kv = dict(l.split(":", 1) for l in open(out) if ":" in l and not l.startswith("#"))
    assert int(kv["traffic_grid_read_bytes"]) == round(1001.0 * 2 * 1024)
    assert int(kv["traffic_grid_write_bytes"]) == round(3000.0 * 1024)
    assert int(kv["traffic_grid_bytes_per_launch"]) == round(1001.0 * 2 * 1024) + round(3000.0 * 1024)
    assert "traffic_frame_bytes_per_launch" not in kv
    assert kv["kernel_source_sha256"].strip() == bench.kernel_source_hash()


def test_pmc_summary_needs_the_calibration_copy(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _pmc_csv(fetch, "FETCH_SIZE", [(bench.TRACKED["grid"], 1000.0)])
    _pmc_csv(write, "WRITE_SIZE", [(bench.TRACKED["grid"], 3000.0)])
    with pytest.raises(SystemExit):
        bench.pmc_summary(str(fetch), str(write), str(tmp_path / "o.txt"), "cmd")


def test_recorded_traffic_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """The committed counter summary counts only for the kernel sources it was taken from."""
    f = tmp_path / "t.txt"
    f.write_text("kernel_source_sha256: %s\ntraffic_grid_bytes_per_launch: 1234\n" % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("grid") == 1234
    assert bench.recorded_traffic("frame") is None
    f.write_text("kernel_source_sha256: 0000000000000000\ntraffic_grid_bytes_per_launch: 1234\n")
    assert bench.recorded_traffic("grid") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.recorded_traffic("grid") is None


def test_stats_summary_lists_every_kernel(tmp_path):
    src = tmp_path / "s.csv"
    with open(src, "w", newline="") as fo:
        w = csv.writer(fo, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["k_a", 10, 1000000, 100000.0, 90.0, 99000, 101000, 1.0])
        w.writerow(["k_b", 10, 100000, 10000.0, 10.0, 9000, 11000, 1.0])
    out = tmp_path / "o.txt"
    bench.stats_summary(str(src), str(out), "the command", "the note")
    text = open(out).read()
    assert "command: the command" in text and "the note" in text
    rows = [l.split() for l in text.splitlines() if l.startswith("k_")]
    assert rows[0][:3] == ["k_a", "10", "100.00"] and rows[1][:3] == ["k_b", "10", "10.00"]


@pytest.mark.parametrize("storage,q,node,pml", [("f64", 37, 592, 656), ("f32", 37, 296, 360),
                                                ("f16", 37, 148, 360), ("f64", 17, 272, 336),
                                                ("f64", 9, 144, 208), ("f32", 9, 72, 136)])
def test_algorithmic_bytes(storage, q, node, pml):
    """q populations read and written per node; a PML node adds Q (compute precision) and the
    four float64 moments, each read and written."""
    assert bench.bytes_per_node(storage, q) == node
    assert bench.pml_extra(storage, q) == pml


def test_kernel_bytes_split_the_step():
    """The step grid's and the frame kernel's algorithmic bytes add up to the step's: the grid
    holds the bulk tiles and phase A's Q update (Q read and written, U^n read per Q node)."""
    g, f, st = bench.kernel_bytes("f64", 37, 1000, 200, 150)
    assert st == 592 * 1200 + 656 * 150
    assert g == 592 * 1000 + (656 - 32) * 150 and f == 592 * 200 + 32 * 150
    g, f, st = bench.kernel_bytes("f64", 37, 1000, 200, 150, fused=False)
    assert g == 592 * 1000 and g + f == st


def test_host_cpu_reports_model_and_cores():
    model, cores = bench.host_cpu()
    assert model and cores and cores >= 1


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


TRACE_COLS = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"]


def _trace_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(TRACE_COLS)
        for name, a, e, g in rows:
            w.writerow(["KERNEL_DISPATCH", name, a, e, g])


def test_gaps_summary_counts_idle_time_between_dispatches(tmp_path):
    """Three steps of [grid, frame] at the group's grid size, preceded by a small run's frame
    kernel: the window runs from the end of the frame before the last three to the end of the
    last; overlapping dispatches count once; idle time is the rest."""
    rows = [("k_frame", 0, 10, 64),                               # another run: smaller grid
            ("k_phase_a_bulk", 20, 60, 999), ("k_frame", 60, 70, 500),   # step 0 (before the window)
            ("k_phase_a_bulk", 75, 115, 999), ("k_frame", 115, 125, 500),
            ("k_advance", 120, 124, 1),                              # inside a busy interval
            ("k_phase_a_bulk", 127, 167, 999), ("k_frame", 170, 180, 500),
            ("k_phase_a_bulk", 180, 220, 999), ("k_frame", 221, 231, 500)]
    rows = [(n, 1000 * a0, 1000 * e0, g) for n, a0, e0, g in rows]   # timestamps in ns, times in us
    src, out = tmp_path / "t.csv", tmp_path / "g.txt"
    _trace_csv(src, rows)
    bench.gaps_summary(str(src), str(out), "cmd", "note", steps=3)
    kv = dict(l.split(":", 1) for l in open(out) if ":" in l and not l.startswith(("#", "command")))
    assert float(kv["wall_us"]) == pytest.approx(231 - 70)
    # idle: 70-75, 125-127, 167-170, 220-221 = 5 + 2 + 3 + 1 = 11 us
    assert float(kv["idle_us"]) == pytest.approx(11)
    assert float(kv["idle_us_per_step"]) == pytest.approx(11 / 3, abs=0.01)


def test_counters_summary_ratios(tmp_path):
    """Busy fractions of the per-CU units are their sums over 32 x GRBM_GUI_ACTIVE (the 8 XCDs'
    sum); wave fractions are over SQ_WAVE_CYCLES; per-wave counts over SQ_WAVES."""
    G = bench.TRACKED["frame"]
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    with open(a, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(COLS)
        for k, (c, v) in enumerate((("GRBM_GUI_ACTIVE", 1000.0), ("SQ_WAVES", 10.0),
                                    ("SQ_WAVE_CYCLES", 400.0), ("SQ_WAIT_INST_ANY", 100.0),
                                    ("SQ_INSTS_VMEM_RD", 150.0))):
            w.writerow([1, 1, G, c, v])
    with open(b, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(COLS)
        for c, v in (("GRBM_GUI_ACTIVE", 1000.0), ("TA_TA_BUSY_sum", 16000.0),
                     ("TCC_HIT_sum", 30.0), ("TCC_MISS_sum", 70.0)):
            w.writerow([1, 1, G, c, v])
    out = tmp_path / "c.txt"
    bench.counters_summary([str(a), str(b)], str(out), "cmd", "note")
    text = open(out).read()
    assert "ratio TA busy" in text and " 0.500" in text.split("ratio TA busy")[1].splitlines()[0]
    assert " 0.250" in text.split("waves waiting on a dependency")[1].splitlines()[0]
    assert " 15.0" in text.split("per wave SQ_INSTS_VMEM_RD")[1].splitlines()[0]
    assert " 0.300" in text.split("L2 hit rate")[1].splitlines()[0]


def test_moment_errors_normalise_by_field_scale():
    import numpy as np
    ref = [np.full((2, 2), 1.0), np.array([[0.1, -0.2], [0.0, 0.05]]), np.zeros((2, 2)),
           np.full((2, 2), 2.0)]
    m = [ref[0] + 1e-9, ref[1] + 2e-9, ref[2] - 4e-9, ref[3] + 2e-9]
    e = bench.moment_errors(m, ref)
    assert e["rho"] == pytest.approx(1e-9)
    assert e["u"] == pytest.approx(4e-9 / 0.2)
    assert e["T"] == pytest.approx(1e-9)
