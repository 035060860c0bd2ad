"""Pins of the oracle's scalar RS propagation (paper: Methods, RS propagation).

Each test checks the oracle against something other than its own formula:
brute-force sums, a derivative identity of the kernel, the paraxial Gaussian
beam closed form, energy conservation, symmetries and the adjoint identity.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import Grid
from tests.conftest import rel_l2


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_kernel_is_minus_dz_of_spherical_wave():
    # H = -(1/2pi) d/dz (e^{ikr}/r): checked by a Richardson-extrapolated
    # central difference of the spherical wave, independent of H's formula.
    wl, z = 650e-9, 3e-3
    k = 2 * math.pi / wl
    X = np.linspace(-1e-3, 1e-3, 7)[None, :]
    Y = np.linspace(-0.7e-3, 0.9e-3, 5)[:, None]
    sph = lambda zz: np.exp(1j * k * np.sqrt(X ** 2 + Y ** 2 + zz ** 2)) / np.sqrt(X ** 2 + Y ** 2 + zz ** 2)
    h = 2e-9
    d1 = (sph(z + h) - sph(z - h)) / (2 * h)
    d2 = (sph(z + 2 * h) - sph(z - 2 * h)) / (4 * h)
    deriv = (4 * d1 - d2) / 3
    H = oracle.rs_kernel(X, Y, z, wl)
    assert rel_l2(H, -deriv / (2 * math.pi)) < 1e-7


def _rs_brute(u, g, wl, z):
    x, y = oracle.coords(g)
    out = np.zeros((g.ny, g.nx), complex)
    for l in range(g.ny):
        for m in range(g.nx):
            acc = 0j
            for i in range(g.ny):
                for j in range(g.nx):
                    acc += u[i, j] * oracle.rs_kernel(x[m] - x[j], y[l] - y[i], z, wl)
            out[l, m] = acc * g.dx * g.dy
    return out


@pytest.mark.parametrize("nx,ny", [(8, 8), (10, 6), (9, 12)])
def test_rs_matches_brute_force_sum(nx, ny):
    g = Grid(nx, ny, 3e-6, 4e-6, 1e-6, -2e-6)
    u = oracle.C128(1) * _rng(nx * ny).standard_normal((ny, nx)) + 1j * _rng(1).standard_normal((ny, nx))
    ref = _rs_brute(u, g, 633e-9, 40e-6)
    assert rel_l2(oracle.rs_propagate(u, g, 633e-9, 40e-6), ref) < 1e-13


def test_rs_sampled_direct_sum_matches_full():
    g = Grid(48, 40, 2e-6, 2.5e-6)
    u = _rng(3).standard_normal((40, 48)) + 1j * _rng(4).standard_normal((40, 48))
    full = oracle.rs_propagate(u, g, 500e-9, 1e-3)
    pix = [(0, 0), (39, 47), (17, 5), (20, 24), (3, 44)]
    got = oracle.rs_at(u, g, 500e-9, 1e-3, pix)
    assert rel_l2(got, np.array([full[p] for p in pix])) < 1e-12


def _gaussian_case():
    # w0 = 50 um, 650 nm, 2 mm window, 512 samples, z = 50 mm (well sampled:
    # z_min = 23.9 mm).  Paraxial corrections are O((lambda/pi w0)^2) ~ 2e-5.
    g = Grid.square(512, 2e-3)
    wl, w0, z = 650e-9, 50e-6, 50e-3
    return g, wl, w0, z


def test_gaussian_beam_width_and_field_closed_form():
    g, wl, w0, z = _gaussian_case()
    assert oracle.rs_sampling_ok(g, wl, z)
    u0 = oracle.gaussian_beam(g, w0)
    u = oracle.rs_propagate(u0, g, wl, z)
    k = 2 * math.pi / wl
    zr = math.pi * w0 ** 2 / wl
    wz = w0 * math.sqrt(1 + (z / zr) ** 2)
    x, y = oracle.coords(g)
    r2 = x[None, :] ** 2 + y[:, None] ** 2
    I = np.abs(u) ** 2
    w_meas = math.sqrt(2 * (I * r2).sum() / I.sum())
    assert abs(w_meas / wz - 1) < 1e-4
    assert abs(wz - 212.857e-6) < 1e-9
    # complex field, paraxial Gaussian beam with Gouy phase (e^{-i w t})
    R = z * (1 + (zr / z) ** 2)
    psi = math.atan(z / zr)
    ref = (w0 / wz) * np.exp(-r2 / wz ** 2) * np.exp(1j * (k * z + k * r2 / (2 * R) - psi))
    core = r2 < (2 * wz) ** 2
    assert rel_l2(u[core], ref[core]) < 2e-4


def test_gaussian_energy_conserved():
    g, wl, w0, z = _gaussian_case()
    u0 = oracle.gaussian_beam(g, w0)
    u = oracle.rs_propagate(u0, g, wl, z)
    e0, e1 = (np.abs(u0) ** 2).sum(), (np.abs(u) ** 2).sum()
    assert abs(e1 / e0 - 1) < 1e-6


def test_flip_and_transpose_symmetry():
    # odd n: the C1 grid is symmetric about the origin
    g = Grid.square(15, 15 * 2e-6)
    u = _rng(5).standard_normal((15, 15)) + 1j * _rng(6).standard_normal((15, 15))
    P = lambda a: oracle.rs_propagate(a, g, 600e-9, 30e-6)
    out = P(u)
    assert rel_l2(P(u[:, ::-1]), out[:, ::-1]) < 1e-13
    assert rel_l2(P(u[::-1, :]), out[::-1, :]) < 1e-13
    assert rel_l2(P(u.T), out.T) < 1e-13


def test_adjoint_dot_product():
    g = Grid(24, 20, 2e-6, 3e-6)
    rng = _rng(7)
    a = rng.standard_normal((20, 24)) + 1j * rng.standard_normal((20, 24))
    b = rng.standard_normal((20, 24)) + 1j * rng.standard_normal((20, 24))
    Aa = oracle.rs_propagate(a, g, 700e-9, 80e-6)
    Ahb = oracle.rs_adjoint(b, g, 700e-9, 80e-6)
    lhs, rhs = np.vdot(b, Aa), np.vdot(Ahb, a)
    assert abs(lhs - rhs) / (np.linalg.norm(Aa) * np.linalg.norm(b)) < 1e-13
    pix = [(0, 0), (19, 23), (7, 11)]
    assert rel_l2(oracle.rs_adjoint_at(b, g, 700e-9, 80e-6, pix), np.array([Ahb[p] for p in pix])) < 1e-12


def test_batch_dimension():
    g = Grid.square(16, 32e-6)
    rng = _rng(8)
    u = rng.standard_normal((3, 16, 16)) + 1j * rng.standard_normal((3, 16, 16))
    out = oracle.rs_propagate(u, g, 500e-9, 50e-6)
    for b in range(3):
        assert rel_l2(out[b], oracle.rs_propagate(u[b], g, 500e-9, 50e-6)) == 0.0


def test_sampling_reading():
    # 2048^2 4 mm at 650 nm: z_min = 23.7 mm
    g = Grid.square(2048, 4e-3)
    assert oracle.rs_sampling_ok(g, 650e-9, 25e-3)
    assert not oracle.rs_sampling_ok(g, 650e-9, 20e-3)
    # 128^2 1 mm at 650 nm, z = 5 mm is undersampled (z_min ~ 24 mm)
    assert not oracle.rs_sampling_ok(Grid.square(128, 1e-3), 650e-9, 5e-3)


def test_kernel_dz_matches_central_difference():
    X, Y = np.meshgrid(np.linspace(-40e-6, 40e-6, 9), np.linspace(-30e-6, 50e-6, 7))
    for z in (20e-6, 3e-3):
        h = 1e-11  # k h ~ 1e-4 rad: the phase e^{ikr} must barely turn over the step
        fd = (oracle.rs_kernel(X, Y, z + h, 600e-9) - oracle.rs_kernel(X, Y, z - h, 600e-9)) / (2 * h)
        an = oracle.rs_kernel_dz(X, Y, z, 600e-9)
        assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()


def test_rs_grad_z_matches_central_difference_of_loss():
    # L(z) = Re <c, RS_z u>: dL/dz from the analytic kernel derivative
    g = Grid(20, 16, 4e-6, 5e-6)
    rng = np.random.default_rng(21)
    u = rng.standard_normal((16, 20)) + 1j * rng.standard_normal((16, 20))
    c = rng.standard_normal((16, 20)) + 1j * rng.standard_normal((16, 20))
    wl, z = 550e-9, 150e-6
    L = lambda zz: float(np.sum(np.real(np.conj(c) * oracle.rs_propagate(u, g, wl, zz))))
    h = 1e-11
    fd = (L(z + h) - L(z - h)) / (2 * h)
    an = oracle.rs_grad_z(u, c, g, wl, z)
    assert abs(fd - an) <= 1e-6 * abs(an)
    both = oracle.rs_grad_z(np.stack([u, 2 * u]), np.stack([c, c]), g, wl, z)
    assert np.allclose(both, [an, 2 * an], rtol=1e-12)
