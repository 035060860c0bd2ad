"""Pins of the oracle's CZT propagation (paper: Methods, CZT with arbitrary
selection and sampling of the region of interest).

Checked against scipy's chirp z-transform, numpy's FFT at the natural window,
the Airy and Gaussian focus closed forms, Parseval, direct sums and the
adjoint identity.
"""
import math

import numpy as np
import pytest
from scipy.signal import czt as scipy_czt
from scipy.special import j1

import oracle
from workloads import Grid
from tests.conftest import rel_l2


def test_one_dimensional_core_matches_scipy_czt():
    # ny = 1 reduces the operator to one zoom DFT along x (y = Y = 0).
    n, m = 37, 23
    gin = Grid(n, 1, 1.7e-6, 1.0, 3e-6, 0.0)
    win = Grid(m, 1, 0.11e-6, 1.0, -0.4e-6, 0.0)
    wl, z = 550e-9, 2e-3
    rng = np.random.default_rng(0)
    u = (rng.standard_normal(n) + 1j * rng.standard_normal(n))[None, :]
    out = oracle.czt_propagate(u, gin, win, wl, z)[0]
    k = 2 * math.pi / wl
    x, _ = oracle.coords(gin)
    X, _ = oracle.coords(win)
    beta = 1 / (wl * z)
    K = np.exp(1j * k * z) * gin.dx * gin.dy / (1j * wl * z)
    a = u[0] * np.exp(1j * k * x ** 2 / (2 * z)) * np.exp(-2j * math.pi * beta * X[0] * x[0])
    # F_p = sum_j a_j exp(-2 pi i beta X_p x_j), X_p = X0 + p dX, x_j = x0 + j dx
    A = np.exp(2j * math.pi * beta * X[0] * gin.dx)
    W = np.exp(-2j * math.pi * beta * gin.dx * win.dx)
    core = scipy_czt(a, m, W, A) * np.exp(-2j * math.pi * beta * x[0] * (X - X[0]))
    ref = K * np.exp(1j * k * X ** 2 / (2 * z)) * core
    assert rel_l2(out, ref) < 1e-12


def test_natural_window_equals_centered_fft():
    n = 64
    gin = Grid.square(n, n * 2e-6)
    wl, z = 600e-9, 5e-3
    d = wl * z / (n * gin.dx)
    win = Grid.square(n, n * d)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    out = oracle.czt_propagate(u, gin, win, wl, z)
    k = 2 * math.pi / wl
    x, y = oracle.coords(gin)
    X, Y = oracle.coords(win)
    Q = np.exp(1j * k * (x[None, :] ** 2 + y[:, None] ** 2) / (2 * z))
    P = np.exp(1j * k * (X[None, :] ** 2 + Y[:, None] ** 2) / (2 * z))
    K = np.exp(1j * k * z) * gin.dx * gin.dy / (1j * wl * z)
    dft = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u * Q)))
    assert rel_l2(out, K * P * dft) < 1e-12
    # Parseval: energy on the natural window equals input energy
    e_in = (np.abs(u) ** 2).sum() * gin.dx * gin.dy
    e_out = (np.abs(out) ** 2).sum() * win.dx * win.dy
    assert abs(e_out / e_in - 1) < 1e-12


def test_airy_focus():
    # uniform disc (a = 0.5 mm) behind a thin lens f = 25 mm, observed at z = f
    a, f, wl = 0.5e-3, 25e-3, 650e-9
    k = 2 * math.pi / wl
    gin = Grid.square(1024, 2e-3)
    x, y = oracle.coords(gin)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    u = np.where(r2 <= a * a, 1.0, 0.0) * np.exp(-1j * k * r2 / (2 * f))
    win = Grid.square(101, 101 * 1e-6)
    I = np.abs(oracle.czt_propagate(u, gin, win, wl, f)) ** 2
    X, Y = oracle.coords(win)
    rho = np.sqrt(X[None, :] ** 2 + Y[:, None] ** 2)
    v = k * a * rho / f
    with np.errstate(invalid="ignore", divide="ignore"):
        airy = np.where(v == 0, 1.0, (2 * j1(v) / v) ** 2)
    Iref = (math.pi * a * a / (wl * f)) ** 2 * airy
    assert abs(I[50, 50] / Iref[50, 50] - 1) < 1e-3
    assert rel_l2(I[50], Iref[50]) < 1e-3
    # first dark ring at 0.6098 lambda f / a
    r0 = 0.6098 * wl * f / a
    assert abs(r0 - 19.8185e-6) < 1e-9


def test_gaussian_focus_complex_closed_form():
    w0, f, wl = 0.2e-3, 25e-3, 650e-9
    k = 2 * math.pi / wl
    gin = Grid.square(512, 2e-3)  # w0 <= L/8
    u = oracle.gaussian_beam(gin, w0, f=f, wavelength=wl)
    win = Grid(64, 48, 0.9e-6, 1.1e-6, 2e-6, -3e-6)
    out = oracle.czt_propagate(u, gin, win, wl, f)
    X, Y = oracle.coords(win)
    rho2 = X[None, :] ** 2 + Y[:, None] ** 2
    ref = (np.exp(1j * k * f) / (1j * wl * f) * np.exp(1j * k * rho2 / (2 * f))
           * math.pi * w0 ** 2 * np.exp(-(math.pi * w0) ** 2 * rho2 / (wl * f) ** 2))
    assert rel_l2(out, ref) < 1e-6


def test_direct_sums_and_adjoint():
    gin = Grid(30, 26, 3e-6, 2.5e-6, 1e-6, 0.5e-6)
    win = Grid(17, 21, 0.4e-6, 0.5e-6, -1e-6, 2e-6)
    wl, z = 480e-9, 1e-3
    rng = np.random.default_rng(2)
    u = rng.standard_normal((26, 30)) + 1j * rng.standard_normal((26, 30))
    gout = rng.standard_normal((21, 17)) + 1j * rng.standard_normal((21, 17))
    out = oracle.czt_propagate(u, gin, win, wl, z)
    pix = [(0, 0), (20, 16), (10, 3)]
    assert rel_l2(oracle.czt_at(u, gin, win, wl, z, pix), np.array([out[p] for p in pix])) < 1e-12
    back = oracle.czt_adjoint(gout, gin, win, wl, z)
    pin = [(0, 0), (25, 29), (11, 7)]
    assert rel_l2(oracle.czt_adjoint_at(gout, gin, win, wl, z, pin), np.array([back[p] for p in pin])) < 1e-12
    lhs, rhs = np.vdot(gout, out), np.vdot(back, u)
    assert abs(lhs - rhs) / (np.linalg.norm(out) * np.linalg.norm(gout)) < 1e-13


def test_rs_and_czt_agree_near_axis():
    # Cross-method sanity: a Gaussian near focus, RS and CZT onto coincident
    # samples; for this narrow angular spectrum the Fresnel residual is tiny.
    wl, w0, f = 650e-9, 0.3e-3, 20e-3
    gin = Grid.square(512, 2e-3)
    u = oracle.gaussian_beam(gin, w0)
    z = 60e-3
    rs = oracle.rs_propagate(u, gin, wl, z)
    win = Grid.square(64, 64 * gin.dx)
    cz = oracle.czt_propagate(u, gin, win, wl, z)
    sl = slice(256 - 32, 256 + 32)
    assert rel_l2(cz, rs[sl, sl]) < 1e-6


def test_czt_grad_z_matches_central_difference_of_loss():
    gi = Grid(24, 20, 3e-6, 3e-6, 2e-6, -1e-6)
    win = Grid(14, 12, 0.8e-6, 0.9e-6, 1e-6, 0.5e-6)
    rng = np.random.default_rng(22)
    u = rng.standard_normal((20, 24)) + 1j * rng.standard_normal((20, 24))
    c = rng.standard_normal((12, 14)) + 1j * rng.standard_normal((12, 14))
    wl, z = 600e-9, 2e-3
    L = lambda zz: float(np.sum(np.real(np.conj(c) * oracle.czt_propagate(u, gi, win, wl, zz))))
    h = 1e-11  # k h ~ 1e-4 rad
    fd = (L(z + h) - L(z - h)) / (2 * h)
    an = oracle.czt_grad_z(u, c, gi, win, wl, z)
    assert abs(fd - an) <= 1e-6 * abs(an)
