"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte table, the conversion of rocprofv3 counter files into HBM bytes per
launch (checked on synthetic counter files with known values), and the CPU
baseline's child processes (on the 64^2 workload)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_kernel_bytes_per_cell():
    n = 256
    N = n ** 3
    # mixed form: residual reads u, d, f and writes u, r (8 + 4 + 8 + 8 + 4 bytes per cell)
    assert bench.kernel_bytes("res", n, 3, True) == 32 * N
    assert bench.kernel_bytes("res", n, 3, False) == 40 * N
    assert bench.kernel_bytes("ls", n, 3, True) == 12 * N
    # spectral passes move the half spectrum (n/2 + 1 complex per x-row) twice
    spec = (n // 2 + 1) * n * n
    assert bench.kernel_bytes("cols_fused", n, 3, True) == 2 * 8 * spec
    assert bench.kernel_bytes("rows_r2c", n, 3, True) == 4 * N + 8 * spec
    assert bench.kernel_bytes("ls_fin", n, 3, True) == 0.0


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_summarize_pmc_scales_by_the_copy(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    res = bench.PASS_KERNELS["res"] + "32>"
    mib = bench.COPY_BYTES / 1024.0  # KiB of the calibration copy
    # the copy reads report half their bytes, writes all of them
    fetch = [(1, copy, "FETCH_SIZE", mib / 2), (2, copy, "FETCH_SIZE", 3.0)]
    write = [(1, copy, "WRITE_SIZE", mib), (2, copy, "WRITE_SIZE", 1.0)]
    # twelve residual launches; the last ten are the timed ones (value 1000 KiB read, 500 written)
    for k in range(12):
        v = 1000.0 if k >= 2 else 99999.0
        fetch.append((10 + k, res + "(psd::Inst const*, psd::Task2 const*)", "FETCH_SIZE", v))
        write.append((10 + k, res + "(psd::Inst const*, psd::Task2 const*)", "WRITE_SIZE", 500.0))
    _write_counters(tmp_path / "f", fetch)
    _write_counters(tmp_path / "w", write)
    out = tmp_path / "traffic.json"
    rec = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(out))
    assert rec["_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["_calibration"]["write_scale"] == pytest.approx(1.0)
    r = rec["c3_256:res"]
    assert r["fetch_bytes"] == 2 * 1000 * 1024
    assert r["write_bytes"] == 500 * 1024
    assert r["bytes_per_launch"] == 2500 * 1024
    assert r["source_hash"] == bench.source_hash()
    assert json.load(open(out)) == rec


def test_source_hash_ignores_comments_only(tmp_path):
    src = os.path.join(ROOT, "paper_1607_01475_amd", "csrc")
    for rel in bench.KERNEL_SOURCES:
        with open(os.path.join(src, rel)) as fh:
            (tmp_path / rel).write_text(fh.read())
    h0 = bench.source_hash(str(tmp_path))
    assert h0 == bench.source_hash()
    k = tmp_path / "psd_kernels.hpp"
    text = k.read_text()
    k.write_text("// a new comment line\n" + text.replace("\n", "  // trailing note\n", 1) + "\n/* block */\n")
    assert bench.source_hash(str(tmp_path)) == h0
    k.write_text(text.replace("PSD_COL_BYTES 128", "PSD_COL_BYTES 64"))
    assert bench.source_hash(str(tmp_path)) != h0


def test_oracle_baseline_children():
    """Single-thread and two side-by-side oracle children on the 64^2 solve:
    both report the oracle's own iteration count and positive rates."""
    out = bench.cpu_baseline("c1", all_cores=False)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    assert "all_cores" not in out
    many, wall = bench.run_oracle_samples("c1", 2)
    assert len(many) == 2 and wall > 0
    assert all(m["iters"] == many[0]["iters"] > 0 for m in many)


def test_trace_summary_separates_early_exits(tmp_path):
    """Kernel-trace summary on synthetic profiler files: launches under the
    early-exit threshold are left out of the working average."""
    stats = tmp_path / "kt_kernel_stats.csv"
    trace = tmp_path / "kt_kernel_trace.csv"

    def write(path, header, rows):
        with open(path, "w", newline="") as fh:
            w = csv.writer(fh)
            w.writerow(header)
            w.writerows(rows)
    write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
          [["void k_res(int)", "3", "244000", "81333", "100.0"]])
    write(trace, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
          [["void k_res(int)", "0", "120000"], ["void k_res(int)", "200000", "320000"],
           ["void k_res(int)", "400000", "404000"]])
    out = tmp_path / "summary.md"
    bench.summarize_trace(str(stats), str(out), "t", "cmd")
    text = out.read_text()
    assert "| `k_res` | 3 | 81.33 | 2 | 120.00 | 120.00 |" in text
