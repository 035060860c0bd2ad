"""Seeded synthetic inputs for the propagation workloads.

This module is shared by the FP64 oracle side and the GPU side. It holds
geometry (grid sizes, pixel pitches, wavelengths, distances) and random
draws only -- no propagation, source or loss arithmetic -- so both sides
consume byte-identical inputs without sharing any of the method's code.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed draw order per workload.  Phases are drawn in float64; FP32 runs cast
them to float32 and the oracle upcasts the *cast* values, so input rounding
is never counted as propagation error.

Workloads (all lengths in metres):

* ``rs_small``   -- 128x128 FP64 scalar RS, 1 mm window, 650 nm, z = 5 mm,
  Gaussian w0 = 200 um times an i.i.d. phase mask.
* ``rs_czt_2048`` -- 2048x2048 scalar RS (z = 25 mm, 4096^2 padded FFT) and
  CZT to the focal plane (z = f = 25 mm, 2048^2 window of 40 um); Gaussian
  w0 = 1 mm, thin lens f = 25 mm, smoothed phase mask.
* ``vector_2048`` -- 2048x2048 radially polarised beam at 532 nm, w0 = 1.2 mm,
  i.i.d. phase mask; VCZT focusing with NA 0.9 onto a 4 um window and VRS
  over 50 mm; 16 finite-difference pixels inside the pupil.
* ``uneven_96``  -- 96 scalar setups with N drawn from {512,...,2048}.
* ``table_32``   -- 32 parameter sets for the two-SLM / two-wave-plate chain.

The paper measures on its own synthetic Gaussian-beam propagations (no
public dataset); these recipes take its shapes and sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterator

import numpy as np

PI = math.pi


@dataclass(frozen=True)
class Grid:
    """Sampling grid: row-major [ny][nx], x fastest.

    Sample (i, j) sits at (cx + (j - nx//2)*dx, cy + (i - ny//2)*dy).
    """

    nx: int
    ny: int
    dx: float
    dy: float
    cx: float = 0.0
    cy: float = 0.0

    @staticmethod
    def square(n: int, extent: float, cx: float = 0.0, cy: float = 0.0) -> "Grid":
        return Grid(n, n, extent / n, extent / n, cx, cy)


def uniform_phase(rng: np.random.Generator, shape) -> np.ndarray:
    """I.i.d. phases uniform in [-pi, pi)."""
    return rng.uniform(-PI, PI, size=shape)


def box5_periodic(a: np.ndarray) -> np.ndarray:
    """5x5 box mean with periodic wrap (input smoothing of a drawn phase map)."""
    acc = np.zeros_like(a)
    for di in range(-2, 3):
        for dj in range(-2, 3):
            acc += np.roll(np.roll(a, di, axis=0), dj, axis=1)
    return acc / 25.0


def random_field(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian test field (real and imaginary parts N(0,1))."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def rs_small(seed: int = 0) -> dict:
    """128^2 FP64 scalar RS case (undersampled by design: parity only)."""
    rng = np.random.default_rng(seed)
    n = 128
    g = Grid.square(n, 1e-3)
    return dict(grid=g, wavelength=650e-9, z=5e-3, w0=200e-6,
                phase=uniform_phase(rng, (n, n)))


def rs_czt_2048(seed: int = 0, n: int = 2048) -> dict:
    """Headline scalar workload: RS over 25 mm and CZT to a 40 um focal window.

    ``n`` may be reduced for parity runs; the pixel pitch then stays 4 mm / n.
    """
    rng = np.random.default_rng(seed)
    g = Grid.square(n, 4e-3)
    win = Grid.square(n, 40e-6)
    phase = box5_periodic(uniform_phase(rng, (n, n)))
    return dict(grid=g, window=win, wavelength=650e-9, z_rs=25e-3, z_czt=25e-3,
                w0=1e-3, f=25e-3, phase=phase)


def vector_2048(seed: int = 0, n: int = 2048) -> dict:
    """Vectorial workload: radial beam, i.i.d. mask, NA 0.9 focusing and VRS."""
    rng = np.random.default_rng(seed)
    extent = 4e-3
    g = Grid.square(n, extent)
    na = 0.9
    win = Grid.square(n, 4e-6)
    phase = uniform_phase(rng, (n, n))
    # 16 finite-difference pixels inside the inscribed pupil disc (integer
    # index geometry with a 2-pixel margin), drawn after the phase map.
    pix = []
    r2max = (n // 2 - 2) ** 2
    while len(pix) < 16:
        i, j = (int(v) for v in rng.integers(0, n, size=2))
        if (i - n // 2) ** 2 + (j - n // 2) ** 2 < r2max and (i, j) not in pix:
            pix.append((i, j))
    return dict(grid=g, window=win, wavelength=532e-9, w0=1.2e-3, na=na,
                f=(extent / 2) / na, z_vrs=50e-3, phase=phase, fd_pixels=pix)


UNEVEN_SIZES = (512, 768, 1024, 1536, 2048)


def uneven_96(seed: int = 0, count: int = 96, sizes=UNEVEN_SIZES) -> Iterator[dict]:
    """Batched uneven scalar setups, drawn lazily in order s = 0..count-1.

    Per setup: N ~ U{sizes}; lambda ~ U[450, 700] nm; z ~ U[5, 100] mm;
    f ~ U[10, 50] mm; phase ~ U[-pi, pi) (N^2, i.i.d.).  Grid 4 mm; RS to z,
    thin lens f, then CZT at z = f onto a 1024^2 window of 40 um.
    """
    rng = np.random.default_rng(seed)
    for s in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        wl = float(rng.uniform(450e-9, 700e-9))
        z = float(rng.uniform(5e-3, 100e-3))
        f = float(rng.uniform(10e-3, 50e-3))
        phase = uniform_phase(rng, (n, n))
        yield dict(index=s, grid=Grid.square(n, 4e-3), window=Grid.square(1024, 40e-6),
                   wavelength=wl, z=z, f=f, w0=1e-3, phase=phase)


def table_32(seed: int = 0, count: int = 32, n: int = 2048) -> Iterator[dict]:
    """Parameter sets for the SLM -> RS -> SLM -> WP -> WP -> focus chain."""
    rng = np.random.default_rng(seed)
    extent = 4e-3
    for s in range(count):
        p1 = uniform_phase(rng, (n, n))
        p2 = uniform_phase(rng, (n, n))
        eta1, th1, eta2, th2 = (float(v) for v in rng.uniform(-PI, PI, size=4))
        yield dict(index=s, grid=Grid.square(n, extent), window=Grid.square(n, 5e-6),
                   wavelength=635e-9, w0=1.2e-3, z=100e-3, na=0.9, f=(extent / 2) / 0.9,
                   phase1=p1, phase2=p2, wp1=(eta1, th1), wp2=(eta2, th2))
