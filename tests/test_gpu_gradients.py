"""Gradients through the hand-written adjoints: torch autograd chains against
the FP64 oracle's adjoint chain and against central finite differences
(paper: Methods, gradient evaluation of the loss with respect to optical
parameters; the phase-mask gradient of the focusing experiments)."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import Grid
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    return lp


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _focus_chain_grad_oracle(vx, vy, phi, g, win, wl, na, f, wfz):
    ux, uy = oracle.modulate(vx, phi), oracle.modulate(vy, phi)
    Ex, Ey, Ez = oracle.vczt_focus(ux, uy, g, win, wl, na, f)
    loss, _, _, (gx, gy, gz) = oracle.spot_loss(win, wl, Ex, Ey, Ez, w_fz=wfz)
    gux, guy = oracle.vczt_focus_adjoint(gx, gy, gz, g, win, wl, na, f)
    return loss, oracle.phase_grad(gux, ux) + oracle.phase_grad(guy, uy)


def _focus_chain_torch(lp, torch, phi_t, g, win, wl, na, f, wfz, w0, dtype):
    from paper_2310_08408_amd.autograd import VCZT, Modulate, SpotLoss
    vx, vy = lp.prop_source_radial(g, w0, dtype=dtype)
    ux, uy = Modulate.apply(vx, phi_t), Modulate.apply(vy, phi_t)
    Ex, Ey, Ez = VCZT.apply(ux, uy, g, win, wl, 0.0, (na, f))
    return SpotLoss.apply(Ex, Ey, Ez, win, wl, wfz).sum()


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_focus_chain_gradient_vs_oracle(lp, kind):
    import torch
    n = 96
    g = Grid.square(n, 4e-3)
    win = Grid.square(48, 48 * 40e-9)
    wl, na, w0 = 532e-9, 0.9, 1.2e-3
    f = 2e-3 / na
    rdt = torch.float32 if kind == "c64" else torch.float64
    dt = torch.complex64 if kind == "c64" else torch.complex128
    phi = np.random.default_rng(0).uniform(-math.pi, math.pi, (1, n, n))
    phi = phi.astype(np.float32).astype(np.float64) if kind == "c64" else phi
    phi_t = torch.tensor(phi, dtype=rdt, device="cuda", requires_grad=True)
    loss = _focus_chain_torch(lp, torch, phi_t, g, win, wl, na, f, 1.0, w0, dt)
    loss.backward()
    vx, vy = oracle.radial_beam(g, w0)
    if kind == "c64":
        vx, vy = (a.astype(np.complex64).astype(np.complex128) for a in (vx, vy))
    ref_loss, ref_grad = _focus_chain_grad_oracle(vx, vy, phi[0], g, win, wl, na, f, 1.0)
    e_loss = abs(float(loss) - ref_loss) / abs(ref_loss)
    e_grad = rel_l2(phi_t.grad.detach().cpu().numpy()[0], ref_grad)
    say(f"focus chain {kind}: loss rel {e_loss:.2e} grad rel-L2 {e_grad:.2e}")
    assert e_grad < (1e-3 if kind == "c64" else 1e-10)
    assert e_loss < (1e-5 if kind == "c64" else 1e-11)


def test_rs_czt_chain_gradcheck_fp64(lp):
    """torch.autograd.gradcheck of SLM -> RS -> SLM -> CZT -> loss on a tiny
    FP64 grid (finite differences against the hand-written adjoints)."""
    import torch
    from paper_2310_08408_amd.autograd import CZT, RS, Modulate, SpotLoss
    g = Grid(12, 10, 20e-6, 20e-6)
    win = Grid(9, 8, 1e-6, 1e-6)
    wl = 600e-9
    v = lp.prop_source_gaussian(g, 80e-6, wl, dtype=torch.complex128)
    p1 = torch.tensor(np.random.default_rng(1).uniform(-1, 1, (1, 10, 12)), device="cuda", requires_grad=True)
    p2 = torch.tensor(np.random.default_rng(2).uniform(-1, 1, (1, 10, 12)), device="cuda", requires_grad=True)

    def fn(a, b):
        u = Modulate.apply(v, a)
        y = RS.apply(u, g, wl, 2e-3)
        y = Modulate.apply(y, b)
        c = CZT.apply(y, g, win, wl, 5e-3)
        return SpotLoss.apply(c, torch.zeros_like(c), None, win, wl, 0.0).sum()

    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        assert torch.autograd.gradcheck(fn, (p1, p2), eps=1e-6, atol=1e-8, rtol=1e-5)


def test_vrs_and_waveplate_gradcheck_fp64(lp):
    import torch
    from paper_2310_08408_amd.autograd import VRS, SpotLoss, WavePlate
    g = Grid(10, 10, 10e-6, 10e-6)
    wl = 550e-9
    rng = np.random.default_rng(3)
    ex = torch.tensor(rng.standard_normal((1, 10, 10)) + 1j * rng.standard_normal((1, 10, 10)), device="cuda",
                      requires_grad=True)
    ey = torch.tensor(rng.standard_normal((1, 10, 10)) + 1j * rng.standard_normal((1, 10, 10)), device="cuda",
                      requires_grad=True)
    eta = torch.tensor(0.4, dtype=torch.float64, device="cuda", requires_grad=True)
    th = torch.tensor(-0.3, dtype=torch.float64, device="cuda", requires_grad=True)

    def fn(a, b, e, t):
        x, y = WavePlate.apply(a, b, e, t)
        X, Y, Z = VRS.apply(x, y, g, wl, 1e-3)
        return SpotLoss.apply(X, Y, Z, g, wl, 0.5).sum()

    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        assert torch.autograd.gradcheck(fn, (ex, ey, eta, th), eps=1e-6, atol=1e-8, rtol=1e-5)


def test_vector_2048_gradient_vs_oracle(lp):
    """Full-size radial focus chain of the vectorial configuration (2048^2
    complex64, 532 nm, NA 0.9 onto a 4 um window, spot-size loss): the FP32
    loss and the whole FP32 gradient map dL/dphi against the FP64 oracle's
    chain (Richards-Wolf integral by zoom matrices, exact adjoint), and the
    16 seed-chosen pupil pixels each against the oracle's own gradient."""
    import os
    import scipy.fft
    import torch
    w = workloads.vector_2048(0)
    g, win, wl, na, f, w0 = w["grid"], w["window"], w["wavelength"], w["na"], w["f"], w["w0"]
    phi32 = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda", requires_grad=True)
    say("2048 focus chain fp32 vs oracle ...")
    loss32 = _focus_chain_torch(lp, torch, phi32, g, win, wl, na, f, 0.0, w0, torch.complex64)
    loss32.backward()
    g32 = phi32.grad.detach().cpu().numpy()[0].astype(np.float64)
    vx, vy = oracle.radial_beam(g, w0)
    phi = phi32.detach().cpu().numpy()[0].astype(np.float64)
    with scipy.fft.set_workers(min(16, os.cpu_count() or 1)):
        ref_loss, ref_grad = _focus_chain_grad_oracle(vx, vy, phi, g, win, wl, na, f, 0.0)
    e_loss = abs(float(loss32) - ref_loss) / abs(ref_loss)
    e_map = rel_l2(g32, ref_grad)
    floor = 1e-3 * np.abs(ref_grad).max()
    e_pix = [abs(g32[i, j] - ref_grad[i, j]) / max(abs(ref_grad[i, j]), floor) for (i, j) in w["fd_pixels"]]
    say(f"  loss {float(loss32):.8e} (oracle {ref_loss:.8e}, rel {e_loss:.2e}); gradient map rel-L2 {e_map:.2e}; "
        f"16 pixels, per-pixel rel max {max(e_pix):.2e}")
    assert e_loss < 1e-5
    assert e_map < 1e-3
    assert max(e_pix) < 1e-3


def test_vector_2048_fd_pixels(lp):
    """Full-size radial focus chain (2048^2 complex64, NA 0.9, 4 um window):
    the hand-written adjoint gradient at 16 seed-chosen pupil pixels against
    central finite differences of the FP64 GPU forward, each pixel against
    its own gradient (with a floor of 1e-3 of the largest), and the whole
    FP32 gradient map against the FP64 GPU gradient map."""
    import torch
    w = workloads.vector_2048(0)
    g, win, wl, na, f, w0 = w["grid"], w["window"], w["wavelength"], w["na"], w["f"], w["w0"]
    phi32 = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda", requires_grad=True)
    say("2048 focus chain fp32 ...")
    loss32 = _focus_chain_torch(lp, torch, phi32, g, win, wl, na, f, 0.0, w0, torch.complex64)
    loss32.backward()
    say("2048 focus chain fp64 ...")
    phi64 = torch.tensor(phi32.detach().cpu().numpy().astype(np.float64), device="cuda", requires_grad=True)
    loss64 = _focus_chain_torch(lp, torch, phi64, g, win, wl, na, f, 0.0, w0, torch.complex128)
    loss64.backward()
    g32 = phi32.grad.detach().cpu().numpy()[0].astype(np.float64)
    g64 = phi64.grad.detach().cpu().numpy()[0]
    e_map = rel_l2(g32, g64)
    say(f"  loss fp32 {float(loss32):.8e} fp64 {float(loss64):.8e}; grad map rel-L2 {e_map:.2e}")
    assert e_map < 1e-3
    h = 1e-4
    floor = 1e-3 * np.abs(g64).max()
    fd_err = []
    with torch.no_grad():
        for (i, j) in w["fd_pixels"]:
            p = phi64.detach().clone()
            p[0, i, j] += h
            lp_ = float(_focus_chain_torch(lp, torch, p, g, win, wl, na, f, 0.0, w0, torch.complex128))
            p[0, i, j] -= 2 * h
            lm_ = float(_focus_chain_torch(lp, torch, p, g, win, wl, na, f, 0.0, w0, torch.complex128))
            fd = (lp_ - lm_) / (2 * h)
            fd_err.append(abs(fd - g32[i, j]) / max(abs(g64[i, j]), floor))
    say(f"  FD vs FP32 adjoint at 16 pixels: max per-pixel |diff| / max(|grad|, 1e-3 max|grad|) = {max(fd_err):.2e}")
    assert max(fd_err) < 1e-3
