"""Pixel-by-pixel evaluators of the oracle's vectorial propagators (direct
sums, used by the full-size GPU checks) against the oracle's whole-field
routines on small grids (paper: Methods, VRS and the high-NA objective).
The VRS evaluator is a direct sum and the whole-field VRS goes through
FFT convolutions, so the two agree only if both sample the kernel the same
way; the focus evaluator sums the pupil for one window pixel at a time."""
import numpy as np

import oracle
import workloads
from workloads import Grid


def _rel(full, at, pix):
    ref = np.array([full[p] for p in pix])
    return np.abs(ref - at).max() / np.abs(full).max()


def test_vrs_at_matches_whole_field():
    rng = np.random.default_rng(0)
    g = Grid(24, 20, 3e-6, 2.5e-6, 1e-6, -0.5e-6)
    ex, ey = workloads.random_field(rng, (20, 24)), workloads.random_field(rng, (20, 24))
    pix = [(0, 0), (19, 23), (7, 11), (12, 3)]
    full = oracle.vrs_propagate(ex, ey, g, 600e-9, 200e-6)
    at = oracle.vrs_at(ex, ey, g, 600e-9, 200e-6, pix)
    assert max(_rel(full[c], at[c], pix) for c in range(3)) < 1e-12
    gs = [workloads.random_field(rng, (20, 24)) for _ in range(3)]
    full = oracle.vrs_adjoint(*gs, g, 600e-9, 200e-6)
    at = oracle.vrs_adjoint_at(*gs, g, 600e-9, 200e-6, pix)
    assert max(_rel(full[c], at[c], pix) for c in range(2)) < 1e-12


def test_focus_at_matches_whole_field():
    rng = np.random.default_rng(1)
    gi = Grid(32, 30, 4e-3 / 32, 4e-3 / 32)
    win = Grid(18, 16, 40e-9, 50e-9, 0.1e-6, 0)
    na = 0.9
    f = (gi.nx * gi.dx / 2) / na
    ex, ey = workloads.random_field(rng, (30, 32)), workloads.random_field(rng, (30, 32))
    pw = [(0, 0), (15, 17), (8, 3)]
    full = oracle.vczt_focus(ex, ey, gi, win, 532e-9, na, f)
    at = oracle.vczt_focus_at(ex, ey, gi, win, 532e-9, na, f, pw)
    assert max(_rel(full[c], at[c], pw) for c in range(3)) < 1e-13
    gs = [workloads.random_field(rng, (16, 18)) for _ in range(3)]
    pi = [(0, 0), (29, 31), (15, 16), (3, 20), (14, 14)]     # corners lie outside the aperture
    full = oracle.vczt_focus_adjoint(*gs, gi, win, 532e-9, na, f)
    at = oracle.vczt_focus_adjoint_at(*gs, gi, win, 532e-9, na, f, pi)
    assert max(_rel(full[c], at[c], pi) for c in range(2)) < 1e-13
    assert at[0][0] == 0 and at[1][1] == 0
