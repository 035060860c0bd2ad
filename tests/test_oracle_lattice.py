"""Pins of the oracle's beam splitter and lattice of building units (paper:
Methods, large-scale search space; Results, large-scale ansatz).

The splitter is pinned by unitarity, its transmit/reflect limits and the
textbook Mach-Zehnder fringe; the lattice wiring by an explicit sum over
monotone light paths; the full objective (units, distances, splitters,
high-NA detectors, density loss, STED, soft minimum) by central finite
differences of its own forward.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import Grid
from tests.conftest import rel_l2


def cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_splitter_is_unitary_and_has_its_limits():
    rng = np.random.default_rng(0)
    a = [cplx(rng, (5, 7)) for _ in range(3)]
    b = [cplx(rng, (5, 7)) for _ in range(3)]
    for alpha in (0.0, 0.3, math.pi / 4, 1.2, math.pi / 2, -2.5):
        c, d = oracle.beam_splitter(a, b, alpha)
        p_in = sum(np.sum(np.abs(x) ** 2) for x in a + b)
        p_out = sum(np.sum(np.abs(x) ** 2) for x in c + d)
        assert abs(p_out / p_in - 1) < 1e-14
    c, d = oracle.beam_splitter(a, b, 0.0)          # T = 1: straight through
    assert all(np.array_equal(x, y) for x, y in zip(c, a)) and all(np.array_equal(x, y) for x, y in zip(d, b))
    c, d = oracle.beam_splitter(a, b, math.pi / 2)  # R = 1: ports swap with a quarter-wave phase
    assert all(np.abs(x - 1j * y).max() < 1e-15 for x, y in zip(c, b))
    assert all(np.abs(x - 1j * y).max() < 1e-15 for x, y in zip(d, a))
    c, d = oracle.beam_splitter(a, None, 0.7)       # dark port b
    assert np.allclose(c[1], math.cos(0.7) * a[1], rtol=0, atol=1e-15)
    assert np.allclose(d[2], 1j * math.sin(0.7) * a[2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("psi", [0.0, 0.4, math.pi / 2, 2.0, math.pi])
def test_mach_zehnder_fringe(psi):
    """Two 50:50 splitters with a phase psi in one arm: the output powers
    are sin^2(psi/2) and cos^2(psi/2) of the input power."""
    a = [np.full((2, 3), 0.6 - 0.8j)]
    c, d = oracle.beam_splitter(a, None, math.pi / 4)
    c = [x * np.exp(1j * psi) for x in c]
    c2, d2 = oracle.beam_splitter(c, d, math.pi / 4)
    assert np.abs(np.abs(c2[0]) ** 2 - math.sin(psi / 2) ** 2).max() < 1e-15
    assert np.abs(np.abs(d2[0]) ** 2 - math.cos(psi / 2) ** 2).max() < 1e-15


def test_splitter_adjoint_and_angle_gradient():
    rng = np.random.default_rng(1)
    a = [cplx(rng, (4, 6)) for _ in range(2)]
    b = [cplx(rng, (4, 6)) for _ in range(2)]
    wc = [cplx(rng, (4, 6)) for _ in range(2)]
    wd = [cplx(rng, (4, 6)) for _ in range(2)]
    alpha = 0.37

    def L(al):  # real linear functional of the outputs: its gradient seeds are wc, wd
        c, d = oracle.beam_splitter(a, b, al)
        return sum(float(np.sum(np.real(np.conj(p) * x))) for p, x in zip(wc + wd, c + d))

    ga, gb, dal = oracle.beam_splitter_adjoint(wc, wd, a, b, alpha)
    h = 1e-6
    fd = (L(alpha + h) - L(alpha - h)) / (2 * h)
    assert abs(fd - dal) <= 1e-8 * max(1.0, abs(dal))
    # input gradients against finite differences in a few entries
    for port, grads in ((a, ga), (b, gb)):
        for comp, (i, j) in ((0, (1, 2)), (1, (3, 5))):
            for unit in (1.0, 1j):
                port[comp][i, j] += h * unit
                lp_ = L(alpha)
                port[comp][i, j] -= 2 * h * unit
                lm = L(alpha)
                port[comp][i, j] += h * unit
                want = grads[comp][i, j].real if unit == 1.0 else grads[comp][i, j].imag
                assert abs((lp_ - lm) / (2 * h) - want) < 1e-8


@pytest.mark.parametrize("R,C", [(1, 1), (2, 2), (2, 3), (3, 3)])
def test_wiring_matches_path_sum_and_conserves_power(R, C):
    rng = np.random.default_rng(R * 10 + C)
    alpha = rng.uniform(-math.pi, math.pi, (R, C))
    nl = oracle.n_links(R, C)
    psi = rng.uniform(-math.pi, math.pi, nl)
    src_amp = cplx(rng, R + C)
    sources = [[np.full((1, 1), s), np.full((1, 1), 0.5 * s)] for s in src_amp]

    def link(l, x):
        return [v * np.exp(1j * psi[l]) for v in x]

    det, _ = oracle.run_lattice(R, C, sources, alpha, link)
    for k in range(R + C):
        want = sum(src_amp[s] * oracle.path_sum(R, C, alpha, psi, s, k) for s in range(R + C))
        assert abs(det[k][0][0, 0] - want) < 1e-13
        assert abs(det[k][1][0, 0] - 0.5 * want) < 1e-13
    p_in = 1.25 * np.sum(np.abs(src_amp) ** 2)
    p_out = sum(abs(d[0][0, 0]) ** 2 + abs(d[1][0, 0]) ** 2 for d in det)
    assert abs(p_out / p_in - 1) < 1e-13


def test_all_transmitting_lattice_keeps_rows_and_columns_apart():
    R, C = 2, 3
    alpha = np.zeros((R, C))
    sources = [None] * (R + C)
    sources[1] = [np.ones((1, 1)), np.zeros((1, 1))]
    det, _ = oracle.run_lattice(R, C, sources, alpha, lambda l, x: x)
    powers = [abs(d[0][0, 0]) ** 2 for d in det]
    assert powers == [0.0, 1.0, 0.0, 0.0, 0.0]


def small_lattice(seed=0, units="all", two_beams=False, comps="ez", R=2, C=2):
    """A tiny lattice: 20 x 18 links grid of 12 um pixels, 8 x 7 detector windows."""
    rng = np.random.default_rng(seed)
    g = Grid(20, 18, 12e-6, 12e-6)
    win = Grid(8, 7, 0.25e-6, 0.25e-6)
    nl = oracle.n_links(R, C)
    unit = np.ones(nl, bool) if units == "all" else np.array([(l % 3) == 0 for l in range(nl)])
    nu = int(unit.sum())
    params = {"unit": unit,
              "phi": rng.uniform(-math.pi, math.pi, (nu, 2, g.ny, g.nx)),
              "wp": rng.uniform(0, math.pi, (nu, 2)),
              "alpha": rng.uniform(0.2, 1.3, (R, C)),
              "z1": rng.uniform(1e-3, 3e-3, nl),
              "z2": np.where(np.arange(nl) % 4 == 1, 0.0, rng.uniform(1e-3, 3e-3, nl))}
    src = oracle.gaussian_beam(g, 60e-6) / math.sqrt(2)
    beams = [{"wavelength": 650e-9, "sources": [[src, src] if s % 2 == 0 else None for s in range(R + C)]}]
    if two_beams:
        beams.append({"wavelength": 532e-9, "sources": [[src, 1j * src] if s % 2 == 1 else None
                                                      for s in range(R + C)]})
    kw = dict(na=0.8, f=2e-3, eps=0.5, comps=comps, beta_sted=1.0, beta_soft=5.0)
    return R, C, g, win, beams, params, kw


@pytest.mark.parametrize("variant", ["ez_all_units", "radial_sted_some_units"])
def test_lattice_gradients_match_finite_differences(variant):
    if variant == "ez_all_units":
        R, C, g, win, beams, params, kw = small_lattice(0)
    else:
        R, C, g, win, beams, params, kw = small_lattice(1, units="some", two_beams=True, comps="radial")
    obj, losses, grads = oracle.lattice_objective(R, C, g, win, beams, params, **kw)
    assert np.isfinite(obj) and obj <= losses.min() + 1e-12

    def f(p):
        return oracle.lattice_objective(R, C, g, win, beams, p, **kw)[0]

    def fd(key, idx, h):
        p1 = {k: np.array(v, copy=True) for k, v in params.items()}
        p2 = {k: np.array(v, copy=True) for k, v in params.items()}
        p1[key][idx] += h
        p2[key][idx] -= h
        return (f(p1) - f(p2)) / (2 * h)

    # distances: small steps, since the selected area of the density loss
    # must not change between the two evaluations
    checks = [("phi", (0, 0, 9, 10), 1e-6), ("phi", (1, 1, 4, 12), 1e-6), ("wp", (0, 0), 1e-6), ("wp", (1, 1), 1e-6),
              ("alpha", (0, 0), 1e-6), ("alpha", (1, 1), 1e-6), ("alpha", (0, 1), 1e-6),
              ("z1", (0,), 2e-10), ("z2", (2,), 2e-10), ("z2", (11,), 2e-10)]
    for key, idx, h in checks:
        want = grads[key][idx]
        got = fd(key, idx, h)
        # relative bar plus the rounding noise of the objective over 2h
        tol = 2e-5 * abs(want) + 3e-14 * max(1.0, abs(obj)) / h
        assert abs(got - want) <= tol, (variant, key, idx, got, want)
