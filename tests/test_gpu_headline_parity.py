"""Whole-field parity of the benchmarked launch against the FP64 oracle.

The headline step at its full size and launch configuration (2048^2
complex64 fields, batch 8, 4096-point persistent RS passes and Bluestein
passes, the fused phase-gradient adjoints), item by item over the whole
field: the SLM field U = V exp(i phi), RS and CZT outputs, the plain
adjoints, and the SLM phase gradient of |Y|^2/2 after the RS adjoint and
after the accumulating CZT adjoint (paper: Methods, RS and CZT propagation
at 2048^2 in Extended Data Fig. 1; gradients with respect to the SLM
phases).  Bars: rel-L2 <= 1e-5 for fields, <= 1e-3 for gradients; each
error is printed.
"""
import os
import sys
import warnings

import numpy as np
import pytest

import oracle
import workloads
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

BATCH = 8
FIELD_TOL, GRAD_TOL = 1e-5, 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def run():
    """The benchmark's inputs and pass sequence on the GPU, intermediate
    results kept per pass (host copies)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    w = workloads.rs_czt_2048(0)
    g, win, wl, zr, zc = w["grid"], w["window"], w["wavelength"], w["z_rs"], w["z_czt"]
    phases = np.stack([w["phase"]] + [workloads.rs_czt_2048(s)["phase"] for s in range(1, BATCH)])
    phi = torch.from_numpy(phases).to(torch.float32).cuda()
    say(f"headline launch: batch {BATCH} x 2048^2 complex64 on the GPU")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        v = lp.prop_source_gaussian(g, w["w0"], wl, lens_f=w["f"], batch=BATCH, dtype=torch.complex64)
        u = lp.prop_modulate(v, phi)
        y_rs = lp.rs_propagate(u, g, wl, zr)
        grad = torch.empty(u.shape, dtype=torch.float32, device="cuda")
        lp.rs_adjoint_phase_grad(y_rs, u, g, wl, zr, grad=grad)
        grad_rs = grad.clone()
        y_czt = lp.czt_propagate(u, g, win, wl, zc)
        lp.czt_adjoint_phase_grad(y_czt, u, g, win, wl, zc, grad=grad, accumulate=True)
        g_rs = lp.rs_adjoint(y_rs, g, wl, zr)
        g_czt = lp.czt_adjoint(y_czt, g, win, wl, zc)
    torch.cuda.synchronize()
    h = lambda t: t.cpu().numpy()
    out = dict(w=w, phi=phases.astype(np.float32).astype(np.float64), u=h(u), y_rs=h(y_rs), y_czt=h(y_czt),
               grad_rs=h(grad_rs), grad=h(grad), g_rs=h(g_rs), g_czt=h(g_czt))
    workers = min(16, os.cpu_count() or 1)
    out["workers"] = workers
    return out


def _oracle_item(run, b):
    """Oracle chain of batch item b (its own FP64 source; the phases as the
    GPU received them)."""
    import scipy.fft
    w = run["w"]
    g, win, wl, zr, zc = w["grid"], w["window"], w["wavelength"], w["z_rs"], w["z_czt"]
    v = oracle.gaussian_beam(g, w["w0"], f=w["f"], wavelength=wl)
    u = oracle.modulate(v, run["phi"][b])
    with scipy.fft.set_workers(run["workers"]):
        y_rs = oracle.rs_propagate(u, g, wl, zr)
        g_rs = oracle.rs_adjoint(y_rs, g, wl, zr)
        y_czt = oracle.czt_propagate(u, g, win, wl, zc)
        g_czt = oracle.czt_adjoint(y_czt, g, win, wl, zc)
    grad_rs = oracle.phase_grad(g_rs, u)
    return dict(u=u, y_rs=y_rs, g_rs=g_rs, y_czt=y_czt, g_czt=g_czt, grad_rs=grad_rs,
                grad=grad_rs + oracle.phase_grad(g_czt, u))


@pytest.mark.parametrize("b", range(BATCH))
def test_headline_whole_field_item(run, b):
    ref = _oracle_item(run, b)
    errs = {k: rel_l2(run[k][b], ref[k]) for k in ("u", "y_rs", "g_rs", "y_czt", "g_czt", "grad_rs", "grad")}
    say(f"item {b}: rel-L2 vs FP64 oracle " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k in ("u", "y_rs", "g_rs", "y_czt", "g_czt"):
        assert errs[k] <= FIELD_TOL, (k, errs[k])
    for k in ("grad_rs", "grad"):
        assert errs[k] <= GRAD_TOL, (k, errs[k])


def test_overlapped_step_equals_serial_step():
    """The benchmarked step runs the CZT forward on a second stream while
    the RS forward and adjoint run on the launch stream; its outputs and
    the accumulated phase gradient equal the serial step's bit for bit
    (same kernels, same accumulation order), over several steps in a row."""
    import torch
    import bench
    import paper_2310_08408_amd as lp
    lp.library()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        w, v, phi = bench.inputs(lp, torch, BATCH, torch.complex64)
        ser = bench.Step(lp, torch, w, v, phi, overlap=False)
        ovl = bench.Step(lp, torch, w, v, phi, overlap=True)
        for k in range(3):
            ser()
            ovl()
            torch.cuda.synchronize()
            assert torch.equal(ser.u, ovl.u), k
            assert torch.equal(ser.grad, ovl.grad), k
            # the CZT output (the serial step writes it over the RS output)
            assert torch.equal(ser.yc, ovl.yc), k
    say(f"overlapped step = serial step over 3 steps (batch {BATCH})")
