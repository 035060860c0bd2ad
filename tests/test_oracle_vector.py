"""Pins of the oracle's vectorial propagators (paper: Methods, VRS and VCZT;
high-NA objective with CZT methods).

VRS/VCZT E_z is pinned by transversality (a tilted beam has E_z/E_x =
-tan(theta)) and by cross-method agreement; the focusing mode by the
Richards-Wolf 1D integrals (Gauss-Legendre with scipy's Bessel functions)
and the radial-beam on-axis zeros; all adjoints by the dot-product identity.
"""
import math

import numpy as np
import pytest
from scipy.special import jv

import oracle
from workloads import Grid
from tests.conftest import rel_l2


def _tilted_beam(g, w0, wl, theta):
    k = 2 * math.pi / wl
    x, _ = oracle.coords(g)
    return oracle.gaussian_beam(g, w0) * np.exp(1j * k * math.sin(theta) * x)[None, :]


def test_vrs_transverse_components_equal_scalar_rs():
    g = Grid.square(32, 32 * 2e-6)
    rng = np.random.default_rng(0)
    ex = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    ey = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    Ex, Ey, Ez = oracle.vrs_propagate(ex, ey, g, 600e-9, 100e-6)
    assert np.array_equal(Ex, oracle.rs_propagate(ex, g, 600e-9, 100e-6))
    assert np.array_equal(Ey, oracle.rs_propagate(ey, g, 600e-9, 100e-6))


def test_vrs_tilted_beam_is_transverse():
    # plane-wave-like beam along (sin t, 0, cos t): E_z / E_x = -tan t
    g = Grid.square(256, 2e-3)
    wl, w0, z, th = 650e-9, 200e-6, 30e-3, 0.02
    ex = _tilted_beam(g, w0, wl, th)
    Ex, Ey, Ez = oracle.vrs_propagate(ex, np.zeros_like(ex), g, wl, z)
    x, y = oracle.coords(g)
    j = int(np.argmin(np.abs(x - z * math.tan(th))))
    i = int(np.argmin(np.abs(y)))
    ratio = Ez[i, j] / Ex[i, j]
    assert abs(ratio + math.tan(th)) < 1e-3 * math.tan(th)
    assert np.abs(Ey).max() < 1e-12 * np.abs(Ex).max()


def test_vrs_symmetry_x_polarised():
    # x-polarised, x-even input: E_z is odd in x and vanishes on the y axis
    g = Grid.square(31, 31 * 3e-6)
    x, y = oracle.coords(g)
    ex = oracle.gaussian_beam(g, 20e-6) * (1 + 0.3 * np.cos(y / 7e-6))[:, None]
    _, _, Ez = oracle.vrs_propagate(ex, np.zeros_like(ex), g, 500e-9, 50e-6)
    assert np.abs(Ez[:, 15]).max() < 1e-13 * np.abs(Ez).max()
    assert rel_l2(Ez[:, ::-1], -Ez) < 1e-13


def test_vczt_free_space_matches_vrs_near_axis():
    g = Grid.square(256, 2e-3)
    # The two differ by the Fresnel residual of the tilted carrier,
    # k z theta^4 / 8 (2.3e-5 rad here); allow twice that.
    wl, w0, z, th = 650e-9, 200e-6, 30e-3, 0.005
    ex = _tilted_beam(g, w0, wl, th)
    ey = 0.5j * oracle.gaussian_beam(g, w0)
    vx, vy, vz = oracle.vrs_propagate(ex, ey, g, wl, z)
    win = Grid.square(64, 64 * g.dx)
    cx, cy, cz = oracle.vczt_propagate(ex, ey, g, win, wl, z)
    sl = slice(128 - 32, 128 + 32)
    tol = 2 * (2 * math.pi / wl) * z * th ** 4 / 8
    assert rel_l2(cx, vx[sl, sl]) < tol
    assert rel_l2(cy, vy[sl, sl]) < 1e-6
    assert rel_l2(cz, vz[sl, sl]) < tol


@pytest.mark.parametrize("op", ["vrs", "vczt", "focus"])
def test_vector_adjoint_dot_product(op):
    rng = np.random.default_rng(3)
    g = Grid(20, 18, 2e-6, 2.2e-6, 0.5e-6, -0.3e-6)
    win = Grid(15, 13, 0.3e-6, 0.35e-6, 0.1e-6, 0.2e-6)
    c = lambda s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    ex, ey = c((18, 20)), c((18, 20))
    if op == "vrs":
        fwd = oracle.vrs_propagate(ex, ey, g, 633e-9, 60e-6)
        gs = [c((18, 20)) for _ in range(3)]
        back = oracle.vrs_adjoint(*gs, g, 633e-9, 60e-6)
    elif op == "vczt":
        fwd = oracle.vczt_propagate(ex, ey, g, win, 633e-9, 60e-6)
        gs = [c((13, 15)) for _ in range(3)]
        back = oracle.vczt_adjoint(*gs, g, win, 633e-9, 60e-6)
    else:
        f = (20 * 2e-6 / 2) / 0.8
        fwd = oracle.vczt_focus(ex, ey, g, win, 633e-9, 0.8, f)
        gs = [c((13, 15)) for _ in range(3)]
        back = oracle.vczt_focus_adjoint(*gs, g, win, 633e-9, 0.8, f)
    lhs = sum(np.vdot(gc, fc) for gc, fc in zip(gs, fwd))
    rhs = np.vdot(back[0], ex) + np.vdot(back[1], ey)
    scale = math.sqrt(sum(np.linalg.norm(f) ** 2 for f in fwd)) * math.sqrt(sum(np.linalg.norm(v) ** 2 for v in gs))
    assert abs(lhs - rhs) / scale < 1e-13


def _rw_integrals(k, f, na, rho, nq=400):
    th_max = math.asin(na)
    t, w = np.polynomial.legendre.leggauss(nq)
    th = 0.5 * th_max * (t + 1)
    w = 0.5 * th_max * w
    ct, st = np.cos(th), np.sin(th)
    a = k * np.asarray(rho)[..., None] * st
    base = np.sqrt(ct) * st
    I00 = (base * (1 + ct) * jv(0, a) * w).sum(-1)
    I01 = (base * st * jv(1, a) * w).sum(-1)
    I02 = (base * (1 - ct) * jv(2, a) * w).sum(-1)
    return I00, I01, I02


def test_focus_matches_richards_wolf_integrals():
    wl, na = 532e-9, 0.9
    k = 2 * math.pi / wl
    n, L = 1023, 4e-3
    g = Grid.square(n, L)
    f = (L / 2) / na
    win = Grid(41, 33, 40e-9, 50e-9, 0.2e-6, -0.1e-6)
    ex = np.ones((n, n), complex)
    Ex, Ey, Ez = oracle.vczt_focus(ex, np.zeros_like(ex), g, win, wl, na, f)
    X, Y = oracle.coords(win)
    XX, YY = np.meshgrid(X, Y)
    rho, phi = np.hypot(XX, YY), np.arctan2(YY, XX)
    I00, I01, I02 = _rw_integrals(k, f, na, rho)
    pre = 1j * k * f / 2 * np.exp(-1j * k * f)
    rx = pre * (I00 + I02 * np.cos(2 * phi))
    ry = pre * I02 * np.sin(2 * phi)
    rz = pre * (-2j) * I01 * np.cos(phi)
    peak = np.abs(rx).max()
    # pupil pixelisation error falls as 1/n (9e-5 at n = 511, 4.6e-5 at 1023)
    assert np.abs(Ex - rx).max() / peak < 2e-4
    assert np.abs(Ey - ry).max() / peak < 2e-4
    assert np.abs(Ez - rz).max() / peak < 2e-4


def test_radial_focus_has_no_transverse_field_on_axis():
    wl, na = 532e-9, 0.9
    g = Grid.square(255, 4e-3)
    f = 2e-3 / na
    ex, ey = oracle.radial_beam(g, 1.2e-3)
    win = Grid.square(9, 9 * 50e-9)
    Ex, Ey, Ez = oracle.vczt_focus(ex, ey, g, win, wl, na, f)
    assert abs(Ex[4, 4]) < 1e-12 * np.abs(Ez).max()
    assert abs(Ey[4, 4]) < 1e-12 * np.abs(Ez).max()
    assert abs(Ez[4, 4]) > 0.5 * np.abs(Ez).max()


def test_radial_beam_peak_is_one():
    g = Grid.square(1001, 4e-3)
    ex, ey = oracle.radial_beam(g, 1.2e-3)
    assert abs(np.sqrt(np.abs(ex) ** 2 + np.abs(ey) ** 2).max() - 1) < 1e-5
