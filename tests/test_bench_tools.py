"""bench.py's trace tools on synthetic rocprofv3 CSV files (no GPU): the
overlap summary of the timed sweeps, checked against hand-counted intervals."""
import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return out.stdout


def test_timeline_summary_counts_overlap_of_the_timed_sweeps_only(tmp_path):
    # one warmup sweep, two timed sweeps and one trailing sweep of two
    # launches each (timestamps in ns).  Timed window [100 us, 400 us]:
    # k_a [100, 200] and k_b [150, 250] overlap for 50 us; then k_a
    # [260, 300] and k_gemm [300, 400]; idle [250, 260].
    us = 1000
    rows = [("void pn::k_a(x)", 0, 10), ("void pn::k_b(x)", 10, 20),
            ("void pn::k_a(x)", 100, 200), ("void pn::k_b(x)", 150, 250),
            ("void pn::k_a(x)", 260, 300), ("void pn::k_gemm<0, 1>(pn::GemmDesc const*)", 300, 400),
            ("void pn::k_a(x)", 500, 510), ("void pn::k_b(x)", 510, 520)]
    p = tmp_path / "run_kernel_trace.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, s, e in rows:
            w.writerow(["KERNEL_DISPATCH", name, s * us * 1000, e * us * 1000])
    out = _run("--timeline-summary", str(p), "2", "2", "1")
    assert "4 launches in 2 timed sweeps, window 300.0 ms (150.0 ms per sweep)" in out
    assert "at least one kernel running: 96.7 %" in out      # 290 of 300
    assert "two or more kernels running: 16.7 %" in out      # 50 of 300
    table = {l.split("|")[1].strip(): (float(l.split("|")[2]), float(l.split("|")[3]))
             for l in out.splitlines() if l.startswith("| k_")}
    # per sweep: summed durations and time running alone
    assert table["k_a"] == (70.0, 45.0)      # (100 + 40) / 2, (50 + 40) / 2
    assert table["k_b"] == (50.0, 25.0)      # 100 / 2, 50 / 2
    assert table["k_gemm"] == (50.0, 50.0)
