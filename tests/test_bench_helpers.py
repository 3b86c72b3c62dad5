"""Host-side helpers of bench.py that summarise profiler output (no GPU, no profiler: synthetic CSV files)."""
from __future__ import annotations

import csv
import io
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def _trace(tmp_path, names_and_durations):
    """A kernel_trace.csv with the kernels back to back (1 us apart), durations in ns."""
    path = tmp_path / "run_kernel_trace.csv"
    t = 1000
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for name, d in names_and_durations:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + d})
            t += d + 1000
    return path


def _call(levels):
    """One clustering call: the offset check, then `levels` levels of (bucket build, two kernels)."""
    ks = [("k_validate_offsets", 10_000)]
    for lv in range(levels):
        ks += [("k_reset_level_counters", 1_000), ("k_enum_grps", 100_000 * (lv + 1)), ("k_apply", 5_000)]
    return ks


def test_level_split_takes_the_last_call(tmp_path):
    first, second = _call(2), _call(3)
    ks = [("k_fill<long>", 2_000)] + first + second + [("k_validate_offsets", 10_000)]  # + the objective check
    _trace(tmp_path, ks)
    out = io.StringIO()
    bench.write_level_split(str(tmp_path), 2, len(ks), out)
    rows = [ln.split() for ln in out.getvalue().splitlines() if not ln.startswith("#")]
    assert [r[0] for r in rows] == ["setup", "0", "1", "2"]
    assert [int(r[1]) for r in rows] == [1, 3, 3, 3]
    assert [float(r[2]) for r in rows] == [0.01, 0.11, 0.21, 0.31]
    assert float(rows[-1][3]) == 0.63  # 0.010 + 0.106 + 0.206 + 0.306


def test_level_split_skips_a_trace_of_another_run(tmp_path):
    ks = _call(2)
    _trace(tmp_path, ks)
    out = io.StringIO()
    bench.write_level_split(str(tmp_path), 1, len(ks) + 1, out)  # the stats count one launch more
    assert out.getvalue() == ""
