"""Host-side checks of the benchmark script: the one-GPU contract and the
rocprofv3 summary helpers that turn counter and trace CSV files into the
tables kept with the profiles (synthetic CSV files, no GPU)."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_short_kernel_names():
    assert bench._short("void sbd::(anonymous namespace)::k_stream<double, 1, 2, 1>(sbd::StreamArgs<double>, "
                        "double const*, double*)") == "k_stream<double,1,2,1>"
    assert bench._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_stats_summary_orders_and_filters(tmp_path):
    p = tmp_path / "k.csv"
    _write(p, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [["sbd::(anonymous namespace)::k_dl_ritz(sbd::DlState*, double*)", "10", "400000", "40000", "20.0"],
            ["void sbd::(anonymous namespace)::k_stream<double, 1, 2, 1>(int)", "2", "1000000", "500000", "50.0"],
            ["void sbd::(anonymous namespace)::k_dl_sub<3>(int)", "10", "100000", "10000", "5.0"]])
    t = bench.stats_summary(str(p)).splitlines()
    assert t[2].startswith("| `k_stream<double,1,2,1>` | 2 | 1.00 | 500.0 | 50.0 |")
    t = bench.stats_summary(str(p), prefix="k_dl").splitlines()
    assert len(t) == 4 and "k_dl_ritz" in t[2] and "k_dl_sub<3>" in t[3]
    t = bench.stats_summary(str(p), prefix="k_stream,k_dl_sub").splitlines()
    assert len(t) == 4 and "k_stream" in t[2] and "k_dl_sub<3>" in t[3]


def test_counters_summary_rates(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void sbd::(anonymous namespace)::k_ab2<double, 1, 10, 1, false>(int)"
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    _write(a, hdr, [[1, k, "TCC_HIT_sum", 300], [1, k, "TCC_MISS_sum", 100],
                    [2, k, "TCC_HIT_sum", 500], [2, k, "TCC_MISS_sum", 100]])
    _write(b, hdr, [[1, k, "TCP_TCC_READ_REQ_sum", 1000], [1, k, "TCP_TCC_READ_REQ_LATENCY_sum", 250000],
                    [1, k, "SQ_INSTS_VALU", 7]])
    t = bench.counters_summary([str(a), str(b)]).splitlines()
    row = t[2].split("|")
    assert "k_ab2<double,1,10,1,false>" in row[1]
    assert row[4].strip() == "400" and row[5].strip() == "100"  # mean hits and misses per dispatch
    assert row[6].strip() == "20.0"                            # miss rate %
    assert row[7].strip() == "250"                             # latency per request
    assert row[8].strip() == "7"


def test_launch_gaps_picks_the_most_frequent_sequence(tmp_path):
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    ns = "void sbd::(anonymous namespace)::"
    names = [ns + "k_transpose<double, 1, false>(int)", ns + "k_stream<double, 1, 2, 1>(int)",
             ns + "k_stream<double, 1, 2, 1>(int)", ns + "k_ab2<double, 1, 10, 1, false>(int)",
             ns + "k_transpose<double, 1, true>(int)"]
    rows, t = [], 0
    for rep in range(3):
        for i, n in enumerate(names):
            gap = 5 if (rep == 2 and i == 3) else 0   # one 5 ns gap in the third sequence
            t += gap
            rows.append([n, t, t + 100])
            t += 100
        t += 10000
    p = tmp_path / "trace.csv"
    _write(p, hdr, rows)
    out = bench.launch_gaps(str(p))
    assert out.startswith("3 sigma sequences of k_transpose<double,1,false> -> k_stream<double,1,2,1>")
    assert "median 0.0 us" in out and "max 0.0 us" in out  # 5 ns rounds to 0.0 us
