"""Pins of the oracle's detector side from the paper: the STED effective
intensity (worked values printed in Methods, STED microscopy), the
threshold-density loss (Methods, loss function) and the soft minimum over
detectors (Methods, exploration of optical topologies)."""
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sted_worked_examples.txt")


def test_sted_worked_examples_from_the_paper():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    closed = {"exp(-1/2)": math.exp(-0.5), "exp(-3/2)": math.exp(-1.5), "(1+exp(-1/2))/2": (1 + math.exp(-0.5)) / 2}
    for beta, ratio, printed, form, dec in rows:
        i_ex = np.array([2.0, 0.7, 13.0])
        got = oracle.sted_intensity(i_ex, float(ratio) * i_ex, float(beta)) / i_ex
        assert np.allclose(got, closed[form], rtol=0, atol=1e-15)
        assert np.all(np.round(got, int(dec)) == float(printed))


def test_sted_limits_stated_in_the_paper():
    i_ex = np.array([0.0, 0.0, 3.0, 3.0, 5.0])
    i_dep = np.array([0.0, 2.0, 0.0, 4.0, 7.0])
    # no excitation -> nothing detected; no depletion -> excitation; beta = 0 -> excitation
    out = oracle.sted_intensity(i_ex, i_dep, 1.0)
    assert out[0] == 0 and out[1] == 0 and out[2] == 3.0
    assert np.allclose(oracle.sted_intensity(i_ex, i_dep, 0.0), i_ex)
    # bounded: 0 <= I_eff <= I_ex
    r = np.random.default_rng(1)
    a, b = r.uniform(0, 5, 1000), r.uniform(0, 5, 1000)
    for beta in (0.0, 0.3, 1.0):
        e = oracle.sted_intensity(a, b, beta)
        assert np.all(e >= 0) and np.all(e <= a + 1e-15)


def test_sted_partials_match_central_differences():
    r = np.random.default_rng(2)
    a, b = r.uniform(0.1, 4, 50), r.uniform(0, 4, 50)
    h = 1e-6
    for beta in (1.0, 0.4):
        pe, pd = oracle.sted_intensity_partials(a, b, beta)
        fe = (oracle.sted_intensity(a + h, b, beta) - oracle.sted_intensity(a - h, b, beta)) / (2 * h)
        fd = (oracle.sted_intensity(a, b + h, beta) - oracle.sted_intensity(a, b - h, beta)) / (2 * h)
        assert np.abs(pe - fe).max() < 1e-8 and np.abs(pd - fd).max() < 1e-8
    # limits at I_ex = 0
    pe, pd = oracle.sted_intensity_partials(np.array([0.0, 0.0]), np.array([1.0, 0.0]), 0.7)
    assert np.allclose(pe, [0.3, 1.0]) and np.allclose(pd, [0.0, -0.7])


def test_density_loss_hand_example():
    # 3x3 detector, eps = 0.5: i_max = 10, threshold 5; selected 10, 8, 6 (5 is not > 5)
    i = np.array([[1.0, 10.0, 2.0], [8.0, 5.0, 0.0], [6.0, 3.0, 4.0]])
    loss, area, ieps, imax, g = oracle.density_loss(i, 0.5)
    assert (area, ieps, imax) == (3.0, 24.0, 10.0)
    assert loss == 3.0 / 24.0
    assert np.array_equal(g != 0, i > 5.0)
    assert np.allclose(g[i > 5.0], -3.0 / 24.0 ** 2)
    # eps = 0: every positive pixel counts
    loss0, area0, ieps0, _, _ = oracle.density_loss(i, 0.0)
    assert (area0, ieps0) == (8.0, 39.0)
    # scaling the intensity scales the loss by its inverse
    assert math.isclose(oracle.density_loss(7.0 * i, 0.5)[0], loss / 7.0, rel_tol=1e-15)


def test_density_loss_seeds_match_central_differences():
    r = np.random.default_rng(3)
    c = lambda: r.standard_normal((9, 11)) + 1j * r.standard_normal((9, 11))
    ex, ey, dx, dy = c(), c(), c(), c()
    for dep in (None, [dx, dy]):
        loss, area, ieps, imax, seeds, seeds_dep = oracle.density_loss_fields([ex, ey], 0.6, dep, 0.8)
        fields = [ex, ey] + (dep or [])
        allseeds = seeds + seeds_dep
        L = lambda fs: oracle.density_loss_fields(fs[:2], 0.6, fs[2:] or None, 0.8)[0]
        h = 1e-7
        checked = 0
        for k, (f, s) in enumerate(zip(fields, allseeds)):
            for (a, b) in [(1, 2), (4, 5), (7, 9), (3, 3)]:
                for unit in (1.0, 1j):
                    fp = [x.copy() for x in fields]; fm = [x.copy() for x in fields]
                    fp[k][a, b] += h * unit; fm[k][a, b] -= h * unit
                    # skip perturbations that change the selection or the maximum
                    if oracle.density_loss_fields(fp[:2], 0.6, fp[2:] or None, 0.8)[1:4:2] != (area, imax) or \
                            oracle.density_loss_fields(fm[:2], 0.6, fm[2:] or None, 0.8)[1:4:2] != (area, imax):
                        continue
                    fd = (L(fp) - L(fm)) / (2 * h)
                    an = s[a, b].real if unit == 1.0 else s[a, b].imag
                    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(loss))
                    checked += 1
        assert checked > 10


def test_softmin_properties():
    l = np.array([0.7, 0.2, 1.5, 0.21])
    v, w = oracle.softmin(l, 1e6)
    assert abs(v - 0.2) < 1e-5                      # large beta -> minimum
    v1, w1 = oracle.softmin(l, 3.0)
    assert v1 <= l.min() and abs(w1.sum() - 1) < 1e-15
    eq, weq = oracle.softmin(np.full(5, 0.4), 2.0)  # equal losses: l - log(n)/beta
    assert abs(eq - (0.4 - math.log(5) / 2.0)) < 1e-15 and np.allclose(weq, 0.2)
    h = 1e-7
    for i in range(4):
        lp, lm = l.copy(), l.copy()
        lp[i] += h; lm[i] -= h
        assert abs((oracle.softmin(lp, 3.0)[0] - oracle.softmin(lm, 3.0)[0]) / (2 * h) - w1[i]) < 1e-7
