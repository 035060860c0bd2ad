#!/usr/bin/env python
"""Text summaries of rocprofv3 CSV output for bench.py runs.

    python bench_profile.py stats DIR [--command TEXT]
        per-kernel calls / average / total time from DIR/*_kernel_stats.csv

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
    import hashlib
    h = hashlib.sha1()
    for f in ("fft_engine.hpp", "fft_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2310_08408_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic}[a.cmd](a)


if __name__ == "__main__":
    main()
