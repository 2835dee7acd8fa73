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
