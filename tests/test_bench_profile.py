"""The rocprofv3 summariser behind profiles/ and the bench's measured
traffic, on small hand-made CSV files (CPU only): the copy-kernel
calibration of FETCH_SIZE / WRITE_SIZE, the per-pass JSON with its source
stamp, and the busy-time union of a kernel trace."""
import argparse
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import bench_profile as bp  # noqa: E402


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, counter, rows):
    _write(os.path.join(d, "run_counter_collection.csv"), ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
           [[k, g, counter, v] for k, g, v in rows])


def test_traffic_calibration_and_stamp(tmp_path, capsys):
    copy = bp.COPY_KERNEL
    rs = "void lp::k_rs_cols_persist<float, lp::Sched<16, 16, 16>, 4, false>(lp::cx<float>*, long)"
    fetch, write = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the copy reads 512 MiB: FETCH_SIZE reads half of that (x2), WRITE_SIZE all of it (x1)
    _counters(fetch, "FETCH_SIZE", [[copy, 131072, 2 ** 18], [rs, 262144, 1000.0], [rs, 262144, 3000.0]])
    _counters(write, "WRITE_SIZE", [[copy, 131072, 2 ** 19], [rs, 262144, 4000.0], [rs, 262144, 4000.0]])
    out = str(tmp_path / "traffic.json")
    bp.cmd_traffic(argparse.Namespace(fetch=fetch, write=write, json=out, command=None))
    text = capsys.readouterr().out
    assert "scale fetch x2.000, write x1.000" in text
    t = json.load(open(out))
    assert set(t) == {"rs_cols"}
    e = t["rs_cols"]
    # mean fetch 2000 KiB x 2 plus write 4000 KiB x 1, per dispatch
    assert e["dispatches"] == 2 and abs(e["bytes_per_launch"] - (2000 * 2 + 4000) * 1024.0) < 1e-6
    assert e["source_sha"] == bench.source_hash()


def test_traffic_needs_the_copy_probe(tmp_path):
    rs = "void lp::k_rs_cols_persist<float, lp::Sched<16, 16, 16>, 4, false>(lp::cx<float>*, long)"
    fetch, write = str(tmp_path / "fetch"), str(tmp_path / "write")
    _counters(fetch, "FETCH_SIZE", [[rs, 262144, 1000.0]])
    _counters(write, "WRITE_SIZE", [[rs, 262144, 4000.0]])
    try:
        bp.cmd_traffic(argparse.Namespace(fetch=fetch, write=write, json=None, command=None))
    except SystemExit as e:
        assert "copy-probe" in str(e)
    else:
        raise AssertionError("a run without the copy probe must be refused")


def test_busy_time_is_the_union_of_kernel_intervals(tmp_path, capsys):
    d = str(tmp_path / "trace")
    # [0,10] and [5,12] overlap (busy 12), gap 12..20, then [20,30]: busy 22 of a 30 ns span
    _write(os.path.join(d, "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["a", 0, 10], ["b", 5, 12], ["c", 20, 30]])
    bp.cmd_busy(argparse.Namespace(dir=d, last=0, command=None))
    text = capsys.readouterr().out
    assert "= 0.7333 of the span" in text and "in 1 gaps" in text
    # sum of durations 10 + 7 + 10 = 27 over 22 busy
    assert "concurrency 1.23" in text
