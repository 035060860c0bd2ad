"""Build libprop.so for gfx950 with hipcc (translation units compiled in parallel).

Usage: python -m paper_2310_08408_amd.build [--jobs N] [--report]
``--report`` prints per-kernel VGPR / scratch / occupancy figures.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libprop.so")

SOURCES = [
    "inst_conv_f32.hip",
    "inst_conv_f64.hip",
    "inst_blue_f32.hip",
    "inst_blue_f64.hip",
    "inst_fft_f32.hip",
    "inst_fft_f64.hip",
    "elementwise.hip",
    "libprop.hip",
]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # the sign of zero is irrelevant here; lets additions of compile-time
    # zeros (pruned transform inputs) fold away
    "-fno-signed-zeros",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, report: bool) -> tuple[str, str]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if report:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    p = subprocess.run(cmd, capture_output=True, text=True)
    log = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{log}")
    return obj, log


def build(jobs: int | None = None, report: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, report), SOURCES))
    objs = [r[0] for r in results]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stdout}\n{p.stderr}")
    os.replace(tmp, LIB)
    if report:
        _print_report("\n".join(r[1] for r in results))
    return LIB


# Host-side AddressSanitizer + UBSan for the ABI layer (argument validation,
# caches, plans) of libprop.hip; device code is built as usual.  Each
# sanitizer flag is scoped to the host compilation.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
SAN_LIB = os.path.join(BUILD, "sanitized", "libprop.so")


def sanitizer_runtime() -> str:
    """The clang ASan runtime (it also carries the UBSan handlers) to preload."""
    base = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(base), reverse=True) if os.path.isdir(base) else []:
        cand = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    raise RuntimeError("clang ASan runtime not found")


def build_host_sanitized() -> str:
    """libprop variant with a sanitized ABI layer, for the host-only ABI tests
    (preload sanitizer_runtime(); the sanitizer runtime is resolved from it,
    not linked in).  Reuses the other translation units of the plain build."""
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if src == "libprop.hip":
            obj = os.path.join(BUILD, "sanitized", "libprop.o")
            cmd = [hipcc(), *FLAGS, *SANITIZE_HOST, "-g", "-c", os.path.join(CSRC, src), "-o", obj]
            p = subprocess.run(cmd, capture_output=True, text=True)
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{p.stderr}")
        elif not os.path.exists(obj):
            _compile(src, False)
        objs.append(obj)
    tmp = SAN_LIB + ".tmp"
    p = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stdout}\n{p.stderr}")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def _print_report(log: str) -> None:
    cur = {}
    rows = []
    for line in log.splitlines():
        if "remark:" not in line:
            continue
        msg = line.split("remark:", 1)[1].strip()
        for key in ("Function Name:", "VGPRs:", "ScratchSize [bytes/lane]:", "Occupancy [waves/SIMD]:", "LDS Size [bytes/block]:"):
            if msg.startswith(key):
                if key == "Function Name:" and cur:
                    rows.append(dict(cur))
                    cur = {}
                cur[key] = msg[len(key):].split("[")[0].strip()
    if cur:
        rows.append(dict(cur))
    for r in rows:
        name = r.get("Function Name:", "?")
        print(f"{r.get('VGPRs:', '?'):>4} vgpr  {r.get('ScratchSize [bytes/lane]:', '?'):>5} scratch  "
              f"occ {r.get('Occupancy [waves/SIMD]:', '?'):>2}  lds {r.get('LDS Size [bytes/block]:', '?'):>6}  {name}")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--report", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.report), file=sys.stderr)
