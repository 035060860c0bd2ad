#!/usr/bin/env python
"""Text summaries of rocprofv3 CSV output for bench.py runs.

    python bench_profile.py stats DIR [--command TEXT]
        per-kernel calls / average / total time from DIR/*_kernel_stats.csv

    python bench_profile.py counters DIR [DIR ...] [--command TEXT]
        SQ counters of the FP32 bench passes (one or more --pmc runs):
        VALU and LDS instructions per wave and per transform point, LDS
        bank-conflict cycles per active LDS cycle, waiting cycles per wave
        cycle, VALU-active cycles per wave cycle.

    python bench_profile.py busy DIR [--last N] [--command TEXT]
        GPU busy time over the window of the last N kernels of a kernel
        trace (union of kernel intervals, idle gaps between them): how much
        launch or dependency overhead a graph replay leaves.

    python bench_profile.py traffic --fetch DIR --write DIR [--json OUT] [--command TEXT]
        HBM bytes per dispatch from two counter runs (FETCH_SIZE, WRITE_SIZE;
        KiB per dispatch), each scaled by what the same counter reads for the
        plain device copy bench.py --copy-probe ends with (64 Mi complex64 =
        512 MiB read + 512 MiB written).  With --json, writes per-pass figures
        keyed by bench.py's pass names, stamped with the hash of the transform
        sources so bench.py can tell when they are stale.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 * 1024 * 1024
COPY_KERNEL = "__amd_rocclr_copyBuffer"

# bench.py pass name -> kernel-name prefix(es) of the FP32 launch it times
# (exact-half shapes run the persistent forms of the row and column passes)
PASS_KERNELS = {
    "rs_rows_fwd": ("void lp::k_rs_rows<float, -1,", "void lp::k_rs_rows_fwd_persist<float,"),
    "rs_cols": ("void lp::k_rs_cols<float,", "void lp::k_rs_cols_persist<float,"),
    "rs_rows_inv": "void lp::k_rs_rows<float, 1,",
    "czt_rows": "void lp::k_bluestein<float, false,",
    "czt_cols": "void lp::k_bluestein<float, true,",
    "modulate": "void lp::k_modulate<float",
    "phase_grad": "void lp::k_phase_grad<float",
}


def short(name: str, width: int = 78) -> str:
    name = name.split("(")[0].replace("void ", "").replace("lp::", "")
    return name if len(name) <= width else name[:width - 3] + "..."


def find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        sys.exit(f"no *{suffix} under {d}")
    return hits[0]


def cmd_stats(a):
    rows = list(csv.DictReader(open(find(a.dir, "kernel_stats.csv"))))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    if a.command:
        print(f"# command: {a.command}")
    print(f"# source: {os.path.basename(find(a.dir, 'kernel_stats.csv'))}; "
          f"all kernels, {total / 1e6:.3f} ms total")
    print(f"{'kernel':80s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>9s} {'%':>6s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        print(f"{short(r['Name']):80s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
              f"{float(r['TotalDurationNs']) / 1e6:9.3f} {100 * float(r['TotalDurationNs']) / total:6.2f}")


def per_dispatch(d: str, counter: str):
    """{(kernel name, grid size): [value per dispatch]} for one counter."""
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(find(d, "counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            out[(r["Kernel_Name"].split("(")[0], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return out


def source_hash() -> str:
    """The stamp bench.py checks before it reports measured traffic."""
    import bench
    return bench.source_hash()


def cmd_traffic(a):
    fetch, write = per_dispatch(a.fetch, "FETCH_SIZE"), per_dispatch(a.write, "WRITE_SIZE")
    mean = lambda v: sum(v) / len(v)
    cf = [mean(v) for k, v in fetch.items() if k[0] == COPY_KERNEL]
    cw = [mean(v) for k, v in write.items() if k[0] == COPY_KERNEL]
    if not cf or not cw:
        sys.exit("no copy-probe dispatch in the counter runs (run bench.py with --copy-probe)")
    f_scale = COPY_BYTES / (cf[-1] * 1024.0)
    w_scale = COPY_BYTES / (cw[-1] * 1024.0)
    if a.command:
        for c in a.command:
            print(f"# command: {c}")
    print(f"# calibration: plain copy of 512 MiB reads FETCH_SIZE {cf[-1]:.4g} KiB, WRITE_SIZE {cw[-1]:.4g} KiB "
          f"-> scale fetch x{f_scale:.3f}, write x{w_scale:.3f}")
    print(f"{'kernel':72s} {'grid':>9s} {'n':>3s} {'fetch_KiB':>11s} {'write_KiB':>11s} {'HBM_MiB':>9s}")
    table = {}
    for key in sorted(set(fetch) | set(write), key=lambda k: -mean(fetch.get(k, [0]))):
        f = mean(fetch[key]) if key in fetch else float("nan")
        w = mean(write[key]) if key in write else float("nan")
        mib = (f * f_scale + w * w_scale) * 1024.0 / 2 ** 20
        table[key] = (len(fetch.get(key, [])), f, w)
        print(f"{short(key[0], 72):72s} {key[1]:9d} {len(fetch.get(key, [])):3d} {f:11.5g} {w:11.5g} {mib:9.2f}")
    if a.json:
        sha = source_hash()
        out = {}
        for name, prefix in PASS_KERNELS.items():
            cands = [k for k in table if k[0].startswith(prefix)]
            if not cands:
                continue
            key = max(cands, key=lambda k: (table[k][0], k[1]))
            n, f, w = table[key]
            out[name] = {"kernel": short(key[0], 200), "grid_size": key[1], "dispatches": n,
                         "fetch_bytes": f * 1024.0 * f_scale, "write_bytes": w * 1024.0 * w_scale,
                         "bytes_per_launch": (f * f_scale + w * w_scale) * 1024.0, "source_sha": sha,
                         "calibration": {"fetch_scale": f_scale, "write_scale": w_scale}}
        with open(a.json, "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
            fh.write("\n")
        print(f"# wrote {os.path.relpath(a.json, ROOT)} ({len(out)} passes, source_sha {sha})")


# transform points (lines x line length) of one batch-8 launch of each FP32
# pass of the 2048^2 bench step: the unit of the per-point instruction counts
BENCH_POINTS = {
    "rs_rows_fwd": 8 * 2048 * 4096,
    "rs_cols": 8 * 4096 * 4096,
    "rs_rows_inv": 8 * 2048 * 4096,
    "czt_rows": 8 * 2048 * 4096,
    "czt_cols": 8 * 2048 * 4096,
}


def cmd_counters(a):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in a.dirs:
        for r in csv.DictReader(open(find(d, "counter_collection.csv"))):
            key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size"]))
            vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    mean = lambda v: sum(v) / len(v) if v else float("nan")
    if a.command:
        for c in a.command:
            print(f"# command: {c}")
    print("# per dispatch (mean over dispatches): VALU/LDS = instructions per wave; per pt = lane instructions per"
          " transform point; bank = conflict cycles per conflict-free LDS cycle, SQ_LDS_BANK_CONFLICT /"
          " (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT); wait = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; valu_act ="
          " SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES (per wave; times the waves per SIMD gives the SIMD's VALU share)")
    print(f"{'pass':12s} {'kernel':66s} {'waves':>8s} {'VALU':>7s} {'LDS':>6s} {'VALU/pt':>8s} {'LDS/pt':>7s} "
          f"{'bank':>6s} {'wait':>6s} {'valu_act':>8s}")
    for name, prefix in PASS_KERNELS.items():
        prefixes = (prefix,) if isinstance(prefix, str) else prefix
        for key in sorted(k for k in vals if k[0].startswith(prefixes)):
            c = {k: mean(v) for k, v in vals[key].items()}
            waves = c.get("SQ_WAVES", float("nan"))
            valu, lds = c.get("SQ_INSTS_VALU", float("nan")), c.get("SQ_INSTS_LDS", float("nan"))
            pts = BENCH_POINTS.get(name)
            per = (lambda x: 64.0 * x / pts) if pts else (lambda x: float("nan"))
            ratio = lambda n, d: c.get(n, float("nan")) / c[d] if c.get(d) else float("nan")
            conf, idx = c.get("SQ_LDS_BANK_CONFLICT", float("nan")), c.get("SQ_LDS_IDX_ACTIVE", float("nan"))
            bank = conf / (idx - conf) if idx and idx > conf else float("nan")
            print(f"{name:12s} {short(key[0], 66):66s} {waves:8.0f} {valu / waves:7.0f} {lds / waves:6.0f} "
                  f"{per(valu):8.2f} {per(lds):7.2f} {bank:6.3f} "
                  f"{ratio('SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES'):6.3f} "
                  f"{ratio('SQ_ACTIVE_INST_VALU', 'SQ_WAVE_CYCLES'):8.3f}")


def cmd_busy(a):
    rows = list(csv.DictReader(open(find(a.dir, "kernel_trace.csv"))))
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    iv = iv[-a.last:] if a.last else iv
    t0, t1 = iv[0][0], max(e for _, e, _ in iv)
    busy, cur_s, cur_e, gaps = 0, iv[0][0], iv[0][1], []
    for st, en, _ in iv[1:]:
        if st > cur_e:
            busy += cur_e - cur_s
            gaps.append(st - cur_e)
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
    busy += cur_e - cur_s
    ksum = sum(e - s for s, e, _ in iv)
    if a.command:
        for c in a.command:
            print(f"# command: {c}")
    span = t1 - t0
    print(f"# window: last {len(iv)} kernels of {len(rows)}; span {span / 1e6:.3f} ms")
    print(f"busy (union of kernel intervals) {busy / 1e6:.3f} ms = {busy / span:.4f} of the span; "
          f"idle {(span - busy) / 1e6:.3f} ms in {len(gaps)} gaps (mean {sum(gaps) / max(len(gaps), 1) / 1e3:.2f} us, "
          f"max {max(gaps or [0]) / 1e3:.2f} us)")
    print(f"sum of kernel durations {ksum / 1e6:.3f} ms (> busy where branches overlap: concurrency "
          f"{ksum / max(busy, 1):.2f})")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--json")
    t.add_argument("--command", action="append")
    b = sub.add_parser("busy")
    b.add_argument("dir")
    b.add_argument("--last", type=int, default=0)
    b.add_argument("--command", action="append")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--command", action="append")
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters, "busy": cmd_busy}[a.cmd](a)


if __name__ == "__main__":
    main()
