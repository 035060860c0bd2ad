"""Pins of the oracle's detector losses, wave plates, SLM phase gradient and
an end-to-end finite-difference check of the adjoint chain (paper: Methods,
gradients of the loss with respect to optical parameters).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import Grid
from tests.conftest import rel_l2


def test_gaussian_spot_second_moment():
    # intensity exp(-2 r^2/w^2) has sigma^2 = w^2 / 2
    win = Grid.square(257, 257 * 10e-9, 0.3e-6, -0.2e-6)
    X, Y = oracle.coords(win)
    w = 0.25e-6
    e = np.exp(-((X[None, :] - 0.31e-6) ** 2 + (Y[:, None] + 0.21e-6) ** 2) / w ** 2)
    _, s2, fz, _ = oracle.spot_loss(win, 1.0, e, np.zeros_like(e))
    assert abs(s2 / (w * w / 2) - 1) < 1e-10
    assert fz == 0.0


def test_spot_translation_invariance():
    win = Grid.square(64, 64 * 20e-9)
    rng = np.random.default_rng(0)
    e = np.zeros((64, 64), complex)
    e[20:30, 18:33] = rng.standard_normal((10, 15)) + 1j * rng.standard_normal((10, 15))
    s_a = oracle.spot_loss(win, 1.0, e, 0 * e)[1]
    s_b = oracle.spot_loss(win, 1.0, np.roll(np.roll(e, 7, 0), -5, 1), 0 * e)[1]
    assert abs(s_a / s_b - 1) < 1e-12


@pytest.mark.parametrize("with_ez", [False, True])
def test_loss_seeds_match_finite_differences(with_ez):
    win = Grid(12, 10, 30e-9, 25e-9, 0.0, 0.0)
    rng = np.random.default_rng(1)
    c = lambda: rng.standard_normal((10, 12)) + 1j * rng.standard_normal((10, 12))
    E = [c(), c(), c()]
    wl, wfz = 532e-9, (0.7 if with_ez else 0.0)

    def L(fields):
        return oracle.spot_loss(win, wl, fields[0], fields[1], fields[2] if with_ez else None, wfz)[0]

    seeds = oracle.spot_loss(win, wl, E[0], E[1], E[2] if with_ez else None, wfz)[3]
    h = 1e-6
    for comp in range(3 if with_ez else 2):
        for (i, j) in [(0, 0), (4, 7), (9, 11)]:
            for part, unit in ((0, 1.0), (1, 1j)):
                Ep = [a.copy() for a in E]; Em = [a.copy() for a in E]
                Ep[comp][i, j] += h * unit; Em[comp][i, j] -= h * unit
                fd = (L(Ep) - L(Em)) / (2 * h)
                an = seeds[comp][i, j].real if part == 0 else seeds[comp][i, j].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_waveplate_properties_and_gradients():
    for eta, th in [(0.3, -1.1), (2.0, 0.4)]:
        J = oracle.waveplate_matrix(eta, th)
        assert np.abs(J.conj().T @ J - np.eye(2)).max() < 1e-15
    assert np.abs(oracle.waveplate_matrix(0.0, 0.7) - np.eye(2)).max() < 1e-15
    hwp = oracle.waveplate_matrix(math.pi, math.pi / 4)
    assert np.abs(hwp - np.array([[0, 1], [1, 0]])).max() < 1e-15
    # quarter-wave plate at 45 deg turns x into circular polarisation
    q = oracle.waveplate_matrix(math.pi / 2, math.pi / 4) @ np.array([1, 0])
    assert abs(abs(q[0]) - abs(q[1])) < 1e-15 and abs(np.angle(q[1] / q[0]) + math.pi / 2) < 1e-12
    rng = np.random.default_rng(2)
    c = lambda: rng.standard_normal((5, 6)) + 1j * rng.standard_normal((5, 6))
    ex, ey, gx, gy = c(), c(), c(), c()

    def L(eta, th):
        ox, oy = oracle.waveplate(ex, ey, eta, th)
        return float(np.sum(np.real(np.conj(gx) * ox + np.conj(gy) * oy)))

    eta, th = 0.9, -0.35
    gex, gey, deta, dth = oracle.waveplate_adjoint(gx, gy, ex, ey, eta, th)
    h = 1e-6
    assert abs((L(eta + h, th) - L(eta - h, th)) / (2 * h) - deta) < 1e-7 * max(1, abs(deta))
    assert abs((L(eta, th + h) - L(eta, th - h)) / (2 * h) - dth) < 1e-7 * max(1, abs(dth))
    # adjoint of the field map
    ox, oy = oracle.waveplate(ex, ey, eta, th)
    lhs = np.vdot(gx, ox) + np.vdot(gy, oy)
    rhs = np.vdot(gex, ex) + np.vdot(gey, ey)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_phase_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((6, 7)) + 1j * rng.standard_normal((6, 7))
    c = rng.standard_normal((6, 7)) + 1j * rng.standard_normal((6, 7))
    phi = rng.uniform(-3, 3, (6, 7))
    L = lambda p: float(np.sum(np.real(np.conj(c) * oracle.modulate(v, p))))
    # for L = Re<c, U>, the gradient seed is g_U = c
    grad = oracle.phase_grad(c, oracle.modulate(v, phi))
    h = 1e-6
    for (i, j) in [(0, 0), (3, 4), (5, 6)]:
        pp, pm = phi.copy(), phi.copy()
        pp[i, j] += h; pm[i, j] -= h
        assert abs((L(pp) - L(pm)) / (2 * h) - grad[i, j]) < 1e-8


def test_focus_chain_gradient_matches_finite_differences():
    # radial beam -> SLM phase -> NA 0.9 focus -> spot size + E_z fraction
    n = 33
    g = Grid.square(n, 4e-3)
    win = Grid.square(17, 17 * 40e-9)
    wl, na = 532e-9, 0.9
    f = 2e-3 / na
    rng = np.random.default_rng(4)
    phi = rng.uniform(-math.pi, math.pi, (n, n))
    vx, vy = oracle.radial_beam(g, 1.2e-3)

    def fwd(p):
        ux, uy = oracle.modulate(vx, p), oracle.modulate(vy, p)
        return ux, uy, oracle.vczt_focus(ux, uy, g, win, wl, na, f)

    ux, uy, (Ex, Ey, Ez) = fwd(phi)
    loss, _, _, (gx, gy, gz) = oracle.spot_loss(win, wl, Ex, Ey, Ez, w_fz=1.0)
    gux, guy = oracle.vczt_focus_adjoint(gx, gy, gz, g, win, wl, na, f)
    grad = oracle.phase_grad(gux, ux) + oracle.phase_grad(guy, uy)
    h = 1e-4
    for (i, j) in [(16, 16), (10, 20), (5, 16), (20, 9)]:
        pp, pm = phi.copy(), phi.copy()
        pp[i, j] += h; pm[i, j] -= h
        Lp = oracle.spot_loss(win, wl, *fwd(pp)[2], w_fz=1.0)[0]
        Lm = oracle.spot_loss(win, wl, *fwd(pm)[2], w_fz=1.0)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[i, j]) <= 1e-6 * np.abs(grad).max()


def test_table_chain_gradients_match_finite_differences():
    """SLM -> RS -> SLM -> WP -> WP -> NA 0.9 objective -> sigma^2/lambda^2 + F_z:
    the oracle's reverse pass against central differences for both phase
    masks and all four retarder parameters."""
    n = 24
    g = Grid.square(n, 24 * 20e-6)
    win = Grid.square(15, 15 * 60e-9)
    wl, z, na = 635e-9, 3e-3, 0.9
    f = (n * 20e-6 / 2) / na
    rng = np.random.default_rng(5)
    v = oracle.gaussian_beam(g, 150e-6) / math.sqrt(2.0)
    p1, p2 = rng.uniform(-math.pi, math.pi, (2, n, n))
    wp1, wp2 = (0.7, -0.4), (1.9, 0.25)
    args = (g, win, wl, z, na, f, 1.0)
    loss, g1, g2, d1, d2 = oracle.table_chain(v, p1, p2, wp1, wp2, *args)
    L = lambda a, b, w1, w2: oracle.table_chain(v, a, b, w1, w2, *args)[0]
    h = 1e-5
    scale = max(np.abs(g1).max(), np.abs(g2).max())
    for (i, j) in [(12, 12), (7, 15), (3, 20)]:
        for which, grad in ((0, g1), (1, g2)):
            pp = [p1.copy(), p2.copy()]; pm = [p1.copy(), p2.copy()]
            pp[which][i, j] += h; pm[which][i, j] -= h
            fd = (L(pp[0], pp[1], wp1, wp2) - L(pm[0], pm[1], wp1, wp2)) / (2 * h)
            assert abs(fd - grad[i, j]) <= 1e-6 * scale
    for plate, d in ((0, d1), (1, d2)):
        for k in range(2):
            wps = [list(wp1), list(wp2)]
            wpp = [list(w) for w in wps]; wpm = [list(w) for w in wps]
            wpp[plate][k] += h; wpm[plate][k] -= h
            fd = (L(p1, p2, *wpp) - L(p1, p2, *wpm)) / (2 * h)
            assert abs(fd - d[k]) <= 1e-6 * max(1.0, abs(d[k]))


@pytest.mark.parametrize("wd", [0.0, 0.05])
def test_adam_step_matches_torch_optim(wd):
    # the library routines (torch.optim.Adam / AdamW on the CPU) as the pin
    import torch
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(6)]
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = (torch.optim.AdamW([t], lr=0.03, weight_decay=wd) if wd else torch.optim.Adam([t], lr=0.03))
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, gk in enumerate(grads, start=1):
        t.grad = torch.tensor(gk, dtype=torch.float64)
        opt.step()
        p, m, v = oracle.adam_step(p, gk, m, v, k, 0.03, weight_decay=wd)
    assert np.abs(p - t.detach().numpy()).max() < 1e-13
