#!/usr/bin/env python
"""Throughput of the propagation gradient hot path on one MI355X.

Workload: 2048^2 complex64 fields on a 4 mm grid at 650 nm (Gaussian beam
w0 = 1 mm, thin lens f = 25 mm, smoothed random phase mask), RS over 25 mm on
a 4096^2 padded transform and CZT to the focal plane onto a 2048^2 window of
40 um.  One step, for a batch of B fields resident in HBM:

    U = V exp(i phi)                       (SLM)
    Y = RS(U),  G = RS^H(Y),  g_phi  = Im(G conj U)     (grad of |Y|^2 / 2)
    Y = CZT(U), G = CZT^H(Y), g_phi += Im(G conj U)

i.e. 2 B gradients (one forward + one adjoint of one propagator on one
field each).  The adjoints write g_phi directly from their last pass
(rs/czt_adjoint_phase_grad).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "2048² RS/CZT fwd+adjoint grads/sec, batched FP32 vs plain FP64; HBM BW %"
HBM_PEAK_GBS = 8000.0
# VALU peak of plain (not packed) FP32 instructions, the only kind the
# kernels use: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The
# published 157.3 TFLOP/s FP32 vector figure counts packed instructions.  A
# probe of independent FMA chains reaches 71.6 TFLOP/s (91% of this peak).
VALU_PEAK_TFLOPS = 78.6


def pass_flops(batch, n=2048, length=4096):
    """Flop model of each FP32 pass of one headline launch: 5 L log2 L per
    transform of length L, times the transforms the pass runs."""
    f = 5.0 * length * math.log2(length)
    return {"rs_rows_fwd": batch * n * f, "rs_cols": batch * 2 * n * 2 * f, "rs_rows_inv": batch * n * f,
            "czt_rows": batch * n * 2 * f, "czt_cols": batch * n * 2 * f, "modulate": 0.0}
BREAKDOWN_STEPS = 10     # untimed steps with every launch traced (per_pass)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def inputs(lp, torch, batch, dtype):
    import numpy as np

    import workloads
    w = workloads.rs_czt_2048(0)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    phases = [w["phase"]] + [workloads.rs_czt_2048(s)["phase"] for s in range(1, batch)]
    phi = torch.from_numpy(np.stack(phases)).to(rdt).cuda()
    v = lp.prop_source_gaussian(w["grid"], w["w0"], w["wavelength"], lens_f=w["f"], batch=batch, dtype=dtype)
    return w, v, phi


class Step:
    """Preallocated buffers and the pass sequence of one gradient step.

    overlap: the CZT forward runs on a second stream (default priority)
    while the RS forward and adjoint run on the launch stream; the CZT
    adjoint, which accumulates into the same gradient, waits for both.  The
    passes are latency-bound, so concurrent kernels fill each other's gaps
    (2.75 -> 2.64 ms per step at batch 8; the gradient is bit-identical to
    the serial order).  Without overlap every pass runs on the launch
    stream in order."""

    def __init__(self, lp, torch, w, v, phi, overlap=False):
        self.lp, self.torch, self.w, self.v, self.phi = lp, torch, w, v, phi
        self.u = torch.empty_like(v)
        self.y = torch.empty_like(v)
        self.yc = torch.empty_like(v) if overlap else self.y
        self.grad = torch.empty(v.shape, dtype=phi.dtype, device=v.device)
        self.side = torch.cuda.Stream() if overlap else None
        self.fork = torch.cuda.Event() if overlap else None

    def __call__(self):
        lp, w, torch = self.lp, self.w, self.torch
        g, win, wl = w["grid"], w["window"], w["wavelength"]
        lp.prop_modulate(self.v, self.phi, out=self.u)
        if self.side is None:
            lp.rs_propagate(self.u, g, wl, w["z_rs"], out=self.y)
            lp.rs_adjoint_phase_grad(self.y, self.u, g, wl, w["z_rs"], grad=self.grad)
            lp.czt_propagate(self.u, g, win, wl, w["z_czt"], out=self.yc)
        else:
            main = torch.cuda.current_stream()
            self.fork.record(main)
            with torch.cuda.stream(self.side):
                self.side.wait_event(self.fork)
                lp.czt_propagate(self.u, g, win, wl, w["z_czt"], out=self.yc)
            lp.rs_propagate(self.u, g, wl, w["z_rs"], out=self.y)
            lp.rs_adjoint_phase_grad(self.y, self.u, g, wl, w["z_rs"], grad=self.grad)
            main.wait_stream(self.side)
        lp.czt_adjoint_phase_grad(self.yc, self.u, g, win, wl, w["z_czt"], grad=self.grad, accumulate=True)


def time_steps(torch, step, steps, warmup):
    """Wall and GPU time per step of `steps` steps between synchronisations,
    and the median of the per-step GPU times (an event between consecutive
    steps on the launch stream)."""
    import statistics
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    gpu = evs[0].elapsed_time(evs[-1]) / 1e3 / steps
    med = statistics.median(evs[i].elapsed_time(evs[i + 1]) for i in range(steps)) / 1e3
    return wall, gpu, med


def source_hash():
    """Hash of the transform sources' code: comments and white space are
    left out, so that a change of documentation keeps the measured traffic."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in ("fft_engine.hpp", "fft_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2310_08408_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the transform sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("source_sha") != source_hash():
        return None
    return e.get("bytes_per_launch")


def rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(reps=3):
    """The FP64 oracle on one 2048^2 field -- RS fwd+adj and CZT fwd+adj with
    the SLM phase gradient, 2 gradients per pass -- timed as the median of
    `reps` passes with all host cores (FFT workers and BLAS threads = nproc)
    and with one thread (about 10 s and 40 s of host work).  Returns the
    record and the oracle's results (RS and CZT forward fields, the summed
    phase gradient) for that field."""
    import statistics

    import scipy.fft
    from threadpoolctl import threadpool_limits

    import oracle
    import workloads
    w = workloads.rs_czt_2048(0)
    g, win, wl = w["grid"], w["window"], w["wavelength"]
    u = oracle.modulate(oracle.gaussian_beam(g, w["w0"], f=w["f"], wavelength=wl), w["phase"])

    def one_pass():
        y = oracle.rs_propagate(u, g, wl, w["z_rs"])
        gr = oracle.rs_adjoint(y, g, wl, w["z_rs"])
        grad = oracle.phase_grad(gr, u)
        yc = oracle.czt_propagate(u, g, win, wl, w["z_czt"])
        gc = oracle.czt_adjoint(yc, g, win, wl, w["z_czt"])
        return y, yc, grad + oracle.phase_grad(gc, u)

    nproc = os.cpu_count() or 1
    times = {}
    for threads in (nproc, 1):
        ts = []
        with threadpool_limits(limits=threads), scipy.fft.set_workers(threads):
            for _ in range(reps):
                t0 = time.perf_counter()
                y, yc, grad = one_pass()
                ts.append(time.perf_counter() - t0)
        times[threads] = statistics.median(ts)
    ref = {"rs_forward": y, "czt_forward": yc, "phase_grad": grad}
    return {"value": 2.0 / times[nproc], "unit": "grads/s", "cores": nproc, "kind": "oracle",
            "sample": f"one 2048^2 field: RS fwd+adj and CZT fwd+adj with the SLM phase gradient (2 gradients) "
                      f"per pass, FP64 numpy/scipy, median of {reps} passes on all {nproc} host threads (FFT "
                      f"workers and BLAS); one thread: {2.0 / times[1]:.4f} grads/s",
            "seconds_per_pass": times[nproc], "single_thread": {"value": 2.0 / times[1], "seconds_per_pass": times[1]},
            "nproc": nproc, "cpu_model": cpu_model(), "reps": reps}, ref


def uneven_leg(lp, torch, reps=5, autotune=True):
    """The 96-setup uneven workload as one plan of chained setups (SLM ->
    RS(z) -> lens f -> CZT at z = f onto a 1024^2 window), forward and
    adjoint as one graph launch (prop_plan_step), by default with lines per workgroup and radix schedules
    picked by the library's autotuner at the plan's first execution (outside
    the timed replays): time per forward+adjoint replay pair,
    setup-gradients/s, the model bytes (per-pass algorithmic reads + writes,
    fused stages included) against HBM peak, and the tuner's choices."""
    import numpy as np

    import workloads
    setups = list(workloads.uneven_96(0, 96, workloads.UNEVEN_SIZES))
    rng = np.random.default_rng(0)
    objs, keep = [], []
    model = 0.0
    t0 = time.perf_counter()
    for w in setups:
        g, win = w["grid"], w["window"]
        v = lp.prop_source_gaussian(g, w["w0"], w["wavelength"])
        phi = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda")
        gy = torch.from_numpy(workloads.random_field(rng, (1, win.ny, win.nx)).astype(np.complex64)).cuda()
        y = torch.empty_like(gy)
        gv, gphi = torch.empty_like(v), torch.empty_like(phi)
        keep += [v, phi, gy, y, gv, gphi]
        objs.append(lp.Setup(lp.PROP_OP_RS_CZT, g, [v], [y], [gy], w["wavelength"], w["z"], window=win,
                             lens_f=w["f"], phase=phi, grad_inputs=[gv], grad_phase=gphi, z2=w["f"]))
        n, mo = g.nx, win.nx
        m = lp.prop_fft_length(2 * n - 1)
        rs = 80.0 * n * n + 8.0 * m * (m // 2 + 1)          # rows, columns (half spectrum), rows
        czt = 8.0 * (n * n + 2.0 * n * mo + mo * mo)        # Bluestein rows, then columns
        stage = 4.0 * n * n + (8.0 + 4.0 + 4.0) * n * n     # phase read; adjoint reads V, phase, writes grad
        model += 2.0 * (rs + czt) + stage
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        plan = lp.Plan(objs, graph=True, autotune=autotune)
        for _ in range(2):
            plan.step()
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.step()
        e1.record()
        e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # one report line per tuned pass shape: "... -> variant v (schedule ..., k per workgroup; timed) ..."
    tuned = [l.split(" -> ")[0].replace("dev 0 ", "") + " -> " + l.split(" -> ")[1].split(";")[0] + ")"
             for l in lp.prop_autotune_report().splitlines() if " -> " in l] if autotune else []
    plan.close()
    del keep
    return {"workload": "uneven96: 96 setups, N in {512,768,1024,1536,2048} drawn from the seed, lambda 450-700 nm, "
                        "RS z 5-100 mm, lens f 10-50 mm, CZT at z=f onto a 1024^2 window of 40 um; complex64, "
                        "FP64 phases; forward+adjoint with SLM phase and input gradients",
            "ms_per_replay_pair": ms, "setup_grads_per_s": 96e3 / ms, "model_bytes": model,
            "hbm_gbs": model / (ms * 1e-3) / 1e9, "hbm_frac": model / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "graph_launches_per_step": 1, "replays": reps, "plan_build_and_warmup_s": build_s,
            "autotuned": autotune, "tuned_shapes": tuned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 96-setup uneven plan leg")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batch 1 / 8 / 32 context timings")
    ap.add_argument("--only-uneven", action="store_true",
                    help="run only the 96-setup uneven plan leg and print its record (profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the 96-setup plan on the built-in schedules (by default the library's autotuner "
                         "picks lines per workgroup and radix schedules at the plan's first execution)")
    ap.add_argument("--no-trace", action="store_true", help="time without per-kernel events")
    ap.add_argument("--serial", action="store_true", help="run every pass of the step on one stream")
    ap.add_argument("--copy-probe", action="store_true",
                    help="finish with a plain 512 MiB device copy (reference for memory counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: libprop shards no work across GPUs (got --gpus {a.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2310_08408_amd as lp
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.only_uneven:
        print(json.dumps(uneven_leg(lp, torch, autotune=not a.no_autotune)), flush=True)
        return

    # ---- batched FP32 path -------------------------------------------------
    log(f"inputs: batch {a.batch} x 2048^2 complex64")
    w, v, phi = inputs(lp, torch, a.batch, torch.complex64)
    step = Step(lp, torch, w, v, phi, overlap=not a.serial)
    t_setup = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log(f"first step (includes kernel-spectrum / chirp setup): {t_setup * 1e3:.1f} ms")
    # The per-pass breakdown and the dominant kernel's roofline come from the
    # serial order of the same step, where each launch has the GPU to itself
    # (event-bracketed durations of kernels that share the GPU with the other
    # stream's kernels measure the sharing, not the kernel).
    kstep = step if a.serial else Step(lp, torch, w, v, phi, overlap=False)
    grads = 2 * a.batch
    trace, live, dom, serial_rec = {}, {}, None, None
    if not a.no_trace:
        for _ in range(a.warmup):
            kstep()
        torch.cuda.synchronize()
        # per-pass breakdown from untimed steps with every launch traced
        lp.prop_trace_enable(True)
        for _ in range(BREAKDOWN_STEPS):
            kstep()
        trace = lp.prop_trace_read()
        lp.prop_trace_enable(False)
        dom = max(trace, key=lambda k: trace[k][1])
        # the timed serial steps trace only the dominant pass (two events per launch)
        lp.prop_trace_only(dom)
        lp.prop_trace_enable(True)
        wall_k, gpu_k, med_k = time_steps(torch, kstep, a.steps, 0)
        live = lp.prop_trace_read()
        lp.prop_trace_enable(False)
        lp.prop_trace_only(None)
        serial_rec = {"ms_per_step": wall_k * 1e3, "value": grads / wall_k, "gpu_ms_per_step_median": med_k * 1e3}
        log(f"serial step: {wall_k * 1e3:.3f} ms/step -> {grads / wall_k:.1f} grads/s")
    if a.serial and serial_rec is not None:
        wall, gpu, med = wall_k, gpu_k, med_k
    else:
        wall, gpu, med = time_steps(torch, step, a.steps, a.warmup)
    if kstep is not step:
        del kstep
    value = grads / wall
    log(f"fp32 batched ({'serial' if a.serial else 'CZT forward overlapped'}): {wall * 1e3:.3f} ms/step wall, "
        f"{gpu * 1e3:.3f} ms/step gpu -> {value:.1f} grads/s")

    per_pass = {}
    flops = pass_flops(a.batch)
    for name, (n, ms, by) in trace.items():
        avg_ms = ms / max(n, 1)
        fl = flops.get(name)
        per_pass[name] = {"launches": n, "avg_ms": avg_ms, "bytes_per_launch": by / max(n, 1),
                          "gbs": (by / max(n, 1)) / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None,
                          "hbm_frac": (by / max(n, 1)) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if avg_ms > 0 else None,
                          "valu_frac": fl / (avg_ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS if fl and avg_ms > 0 else None,
                          "share": ms / max(sum(t[1] for t in trace.values()), 1e-12)}
    roofline = None
    if dom in live:
        n, ms, by = live[dom]
        avg_ms, bpl = ms / max(n, 1), by / max(n, 1)
        gbs = bpl / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(dom), "kernel": dom,
                    "bytes_per_launch": bpl, "avg_ms": avg_ms, "launches": n,
                    "step": "serial: every pass on one stream, each launch alone on the GPU"}
        if flops.get(dom):
            tf = flops[dom] / (avg_ms * 1e-3) / 1e12
            roofline["valu_frac"] = tf / VALU_PEAK_TFLOPS
            roofline["valu"] = {"bound": "alu", "achieved": tf, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": tf / VALU_PEAK_TFLOPS, "flops_per_launch": flops[dom],
                                "model": "5 L log2 L per length-L transform; plain (not packed) FP32 VALU peak"}
    total_model_bytes = sum(t[2] for t in trace.values()) / BREAKDOWN_STEPS
    step_frac = total_model_bytes / wall / 1e9 / HBM_PEAK_GBS if trace else None

    # ---- errors vs the GPU FP64 path, and its plain single-field timing ----
    log("fp64 single-field path")
    w64, v64, phi64 = inputs(lp, torch, 1, torch.complex128)
    step64 = Step(lp, torch, w64, v64, phi64)
    step64()
    torch.cuda.synchronize()
    errs = {}
    # FP32 results come from the same batched launches the timed step uses
    # (item 0 of the batch), so every FP32 kernel launch has one shape.
    g, win, wl = w["grid"], w["window"], w["wavelength"]
    y32 = lp.rs_propagate(step.u, g, wl, w["z_rs"])
    y64 = lp.rs_propagate(step64.u, g, wl, w["z_rs"])
    errs["rs_forward"] = rel(y32[:1].to(torch.complex128), y64)
    errs["rs_adjoint"] = rel(lp.rs_adjoint(y32, g, wl, w["z_rs"])[:1].to(torch.complex128),
                             lp.rs_adjoint(y64, g, wl, w["z_rs"]))
    c32 = lp.czt_propagate(step.u, g, win, wl, w["z_czt"])
    c64 = lp.czt_propagate(step64.u, g, win, wl, w["z_czt"])
    errs["czt_forward"] = rel(c32[:1].to(torch.complex128), c64)
    errs["czt_adjoint"] = rel(lp.czt_adjoint(c32, g, win, wl, w["z_czt"])[:1].to(torch.complex128),
                              lp.czt_adjoint(c64, g, win, wl, w["z_czt"]))
    errs["phase_grad"] = rel(step.grad[:1].to(torch.float64), step64.grad)
    log("rel-L2 of FP32 results vs the FP64 GPU path:", {k: f"{v:.2e}" for k, v in errs.items()})
    wall64, _, _ = time_steps(torch, step64, a.fp64_steps, 1)
    value64 = 2 / wall64
    log(f"fp64 single field: {wall64 * 1e3:.3f} ms/step -> {value64:.1f} grads/s")

    # achievable HBM rate for context: a plain 512 MiB device-to-device copy
    # (reads 512 MiB, writes 512 MiB), best of 10, after the timed region
    src = torch.empty(64 * 1024 * 1024, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    copy_gbs = 2 * src.numel() * 8 / (best * 1e-3) / 1e9
    del src, dst
    log(f"device copy of 512 MiB: {copy_gbs:.0f} GB/s")

    # the same step at the other batch sizes of the protocol (B in {1, 8, 32});
    # context only: the headline stays at --batch
    sweep = None
    if not a.no_sweep:
        sweep = {}
        for b in (1, 8, 32):
            if b == a.batch:
                continue
            wb, vb, phib = inputs(lp, torch, b, torch.complex64)
            sb = Step(lp, torch, wb, vb, phib, overlap=not a.serial)
            wall_b, _, med_b = time_steps(torch, sb, 20, 5)
            sweep[str(b)] = {"ms_per_step": wall_b * 1e3, "gpu_ms_per_step_median": med_b * 1e3,
                             "value": 2 * b / wall_b, "unit": "grads/s"}
            log(f"batch {b}: {wall_b * 1e3:.3f} ms/step -> {2 * b / wall_b:.1f} grads/s")
            del sb, vb, phib
        torch.cuda.empty_cache()

    uneven = None
    if not a.no_uneven:
        log("uneven 96-setup plan ...")
        uneven = uneven_leg(lp, torch, autotune=not a.no_autotune)
        log(f"uneven 96: {uneven['ms_per_replay_pair']:.2f} ms per forward+adjoint replay pair, "
            f"{uneven['setup_grads_per_s']:.0f} setup-gradients/s, {uneven['hbm_frac']:.3f} of HBM peak")

    cpu, errs_oracle = None, None
    if not a.no_cpu:
        import numpy as np
        log("cpu baseline (FP64 oracle) ...")
        cpu, ref = cpu_baseline()
        log(f"cpu baseline: {cpu['value']:.4f} grads/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.4f} on one ({cpu['cpu_model']})")
        # item 0 of the batch is the oracle's field: FP32 results against it
        got = {"rs_forward": y32[0], "czt_forward": c32[0], "phase_grad": step.grad[0]}
        errs_oracle = {}
        for k, t in got.items():
            x = t.detach().cpu().numpy().astype(np.complex128)
            errs_oracle[k] = float(np.linalg.norm(x - ref[k]) / np.linalg.norm(ref[k]))
        log("rel-L2 of FP32 results (item 0) vs the FP64 oracle:", {k: f"{v:.2e}" for k, v in errs_oracle.items()})

    out = {
        "metric": METRIC, "value": value, "unit": "grads/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rs_czt_2048: 2048^2 complex64 fields, 4 mm grid, 650 nm; RS z=25 mm (4096^2 padded) "
                               "+ CZT z=f=25 mm onto a 2048^2 40 um window; SLM phase gradient of |Y|^2/2",
                   "batch": a.batch, "grads_per_step": grads,
                   "streams": 1 if a.serial else 2},
        "roofline": roofline,
        "serial_step": serial_rec,
        "cpu_baseline": cpu,
        "hbm_frac_step": step_frac,
        "hbm_copy": {"gbs": copy_gbs, "bytes": 2 * 512 * 2 ** 20, "what": "512 MiB device-to-device copy, best of 10",
                     "dominant_frac_of_copy": (roofline["achieved"] / copy_gbs) if roofline else None},
        "fp64_single": {"value": value64, "unit": "grads/s", "ms_per_step": wall64 * 1e3,
                        "speedup_fp32_batched": value / value64},
        "errors_vs_fp64": errs,
        "errors_vs_oracle": errs_oracle,
        "per_pass": per_pass,
        "uneven96": uneven,
        "batch_sweep": sweep,
        "gpu_ms_per_step": gpu * 1e3,
        "gpu_ms_per_step_median": med * 1e3,
        "first_step_ms": t_setup * 1e3,
    }
    print(json.dumps(out), flush=True)
    if a.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
