"""Lattice of beam splitters joined by building units: the paper's large-scale
ansatz (Results, general virtual optical setup for large-scale discovery;
Methods, the large-scale search space and the discovery experiments).

The paper names the parts -- building units made of a super-SLM and a wave
plate a distance apart, free propagation, beam splitters with [T, R]
ratios, several sources and high-NA detectors, a loss per detector combined
by a smooth minimum -- and their counts for the 3 x 3 grid, but not how they
are wired.  This module takes the following layout:

* an R x C grid of splitters; the light of row r enters splitter (r, 0)
  from the left, that of column c enters splitter (0, c) from the top;
  every splitter sends its port c to the right and its port d downwards,
  and the grid ends in R + C detectors (right ends of the rows, then bottom
  ends of the columns);
* a splitter mixes its ports with one angle alpha (T = cos^2, R = sin^2):
  c = cos a + i sin b, d = i sin a + cos b, on each field component;
* every link (source -> splitter, splitter -> splitter, splitter ->
  detector) may hold a building unit -- super-SLM (phases on E_x and E_y),
  propagation over z1, wave plate -- and then propagates over its own z2;
* propagation between elements carries the transverse field: the x and y
  components of vectorial RS are scalar RS of E_x and E_y, and E_z is only
  formed by the detectors' objectives (Richards-Wolf focusing), where the
  loss needs it;
* beams of different wavelengths run through the lattice separately with
  the same parameters; a second beam acts as the STED depletion beam.

Links are numbered: horizontal link (r, j) (j = 0..C) is r (C + 1) + j,
vertical link (i, c) (i = 0..R) is R (C + 1) + c (R + 1) + i.  Every
element is a libprop call behind a torch.autograd.Function, so the backward
pass runs the hand-written adjoints and keeps, per element, only what its
adjoint needs (the linear propagators keep nothing but the input of a
differentiated distance).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from .autograd import (CZT, RS, VCZT, BeamSplitter, BeamSplitterPair, DensityLoss, Modulate,  # noqa: F401
                       ModulatePair, SoftMin, WavePlates, WavePlatesPair)

COMPONENTS = {"ez": (2,), "radial": (0, 1), "total": (0, 1, 2)}


def n_links(R: int, C: int) -> int:
    return R * (C + 1) + C * (R + 1)


def h_link(R: int, C: int, r: int, j: int) -> int:
    return r * (C + 1) + j


def v_link(R: int, C: int, i: int, c: int) -> int:
    return R * (C + 1) + c * (R + 1) + i


@dataclass
class LatticeParams:
    """Optimisable parameters of one batch of lattices (batch B).

    phi[k]   = (phi_x, phi_y), real [B, ny, nx] each, super-SLM of unit k;
    wp[k]    = float64 [B, 2] (eta, theta) of unit k's wave plate;
    alpha    = float64 [R * C, B] splitter angles, row-major over (r, c);
    z1[l], z2[l] = float or 0-d float64 tensor per link (z1 used by units).
    """
    phi: list = field(default_factory=list)
    wp: list = field(default_factory=list)
    alpha: torch.Tensor = None
    z1: list = field(default_factory=list)
    z2: list = field(default_factory=list)

    def tensors(self):
        out = [t for pair in self.phi for t in pair] + list(self.wp) + [self.alpha]
        out += [z for z in list(self.z1) + list(self.z2) if isinstance(z, torch.Tensor)]
        return out


def _host_distances(p: LatticeParams):
    """Host values of (z1, z2) per link.  The distances may be 0-d device
    tensors; they are read back together in one transfer, since every
    separate read waits for the device queue to drain."""
    zs = list(p.z1) + list(p.z2)
    ts = [z for z in zs if isinstance(z, torch.Tensor)]
    vals = iter(torch.stack([t.detach().to(torch.float64).reshape(()) for t in ts]).cpu().tolist() if ts else [])
    host = [next(vals) if isinstance(z, torch.Tensor) else float(z) for z in zs]
    return host[:len(p.z1)], host[len(p.z1):]


class Lattice:
    """R x C splitter lattice with building units on the links in `unit`
    (a sequence of nlinks booleans), high-NA detectors (na, f) onto
    `window`, and the density loss of components `comps` ('ez', 'radial',
    'total') with threshold eps, STED efficiency beta_sted, and a smooth
    minimum with sharpness beta_soft over the R + C detectors."""

    def __init__(self, R, C, grid, window, na, f, unit, comps="ez", eps=0.7, beta_sted=1.0, beta_soft=10.0):
        self.R, self.C = R, C
        self.grid, self.window = grid, window
        self.lens = (na, f)
        self.nl = n_links(R, C)
        self.unit = [bool(u) for u in unit]
        if len(self.unit) != self.nl:
            raise ValueError(f"unit mask needs {self.nl} entries")
        self.unit_index, k = [], 0
        for u in self.unit:
            self.unit_index.append(k if u else -1)
            k += int(u)
        self.n_units = k
        self.sel = COMPONENTS[comps]
        self.eps, self.beta_sted, self.beta_soft = eps, beta_sted, beta_soft

    # ------------------------------------------------------------ elements
    # Inside the lattice a port's field is one stacked tensor [2, B, ny, nx]
    # (E_x, E_y): both components propagate in one RS call over 2B planes.
    def _rs(self, s, wl, z, zv):
        two, b, ny, nx = s.shape
        return RS.apply(s.reshape(two * b, ny, nx), self.grid, wl, z, zv).reshape(s.shape)

    def _link(self, l, s, wl, p, zh):
        if s is None:
            return None
        z1, z2 = zh[0][l], zh[1][l]
        if self.unit[l]:
            k = self.unit_index[l]
            s = ModulatePair.apply(s, p.phi[k][0], p.phi[k][1])
            s = self._rs(s, wl, p.z1[l], z1)
            s = WavePlatesPair.apply(s, p.wp[k])
        if z2 > 0:
            s = self._rs(s, wl, p.z2[l], z2)
        return s

    @staticmethod
    def _split(a, b, alpha):
        if a is None and b is None:
            return None, None
        return BeamSplitterPair.apply(alpha, a, b)

    def detector_fields(self, sources, wl, p, zh=None):
        """Transverse fields arriving at the R + C detectors for one beam;
        sources: R + C entries (ex, ey) [B, ny, nx] or None (dark); zh: the
        host values of p's distances (read from p when not given)."""
        R, C = self.R, self.C
        if len(sources) != R + C:
            raise ValueError(f"need {R + C} sources")
        if zh is None:
            zh = _host_distances(p)
        stacked = [None if s is None else torch.stack([s[0], s[1]]) for s in sources]
        h = {(r, 0): stacked[r] for r in range(R)}
        v = {(0, c): stacked[R + c] for c in range(C)}
        for r in range(R):
            for c in range(C):
                a = self._link(h_link(R, C, r, c), h[(r, c)], wl, p, zh)
                b = self._link(v_link(R, C, r, c), v[(r, c)], wl, p, zh)
                h[(r, c + 1)], v[(r + 1, c)] = self._split(a, b, p.alpha[r * C + c])
        det = [self._link(h_link(R, C, r, C), h[(r, C)], wl, p, zh) for r in range(R)]
        det += [self._link(v_link(R, C, R, c), v[(R, c)], wl, p, zh) for c in range(C)]
        return [None if d is None else tuple(d.unbind(0)) for d in det]

    def forward(self, beams, p: LatticeParams):
        """beams: list of 1 or 2 dicts {"wavelength", "sources"}; the second
        is the STED depletion beam.  Returns (objective [B] float64,
        per-detector losses [B, R + C] float64), differentiable in p."""
        focused = []
        zh = _host_distances(p)
        for beam in beams:
            wl = beam["wavelength"]
            det = self.detector_fields(beam["sources"], wl, p, zh)
            outs = []
            for k, d in enumerate(det):
                if d is None:
                    # no source of this beam reaches detector k: allowed
                    # for the depletion beam (no depletion), not for the
                    # excitation beam (its loss would be undefined)
                    if not focused:
                        raise ValueError(f"no light reaches detector {k}")
                    outs.append(None)
                    continue
                outs.append(VCZT.apply(d[0], d[1], self.grid, self.window, wl, 0.0, self.lens))
            focused.append(outs)
        losses = []
        for k in range(self.R + self.C):
            ex = [focused[0][k][c] for c in self.sel]
            dep = [focused[1][k][c] for c in self.sel] if len(focused) > 1 and focused[1][k] is not None else []
            losses.append(DensityLoss.apply(len(ex), self.eps, self.beta_sted, *ex, *dep))
        losses = torch.stack(losses, dim=-1)
        return SoftMin.apply(losses, self.beta_soft), losses

    # -------------------------------------------------------------- set-up
    def random_params(self, batch, seed=0, real_dtype=torch.float32, device="cuda", z_range=(5e-3, 5e-2),
                      requires_grad=True):
        """Parameters drawn from a seeded generator on the host: phases
        uniform in [0, 1) (the paper initialises its optical parameters
        between 0 and 1), wave plates and splitter angles uniform in [0, 1),
        distances uniform in z_range."""
        gen = torch.Generator().manual_seed(seed)
        ny, nx = self.grid.ny, self.grid.nx

        def u(*shape, dt=torch.float64):
            return torch.rand(*shape, generator=gen, dtype=torch.float64).to(dt).to(device).requires_grad_(
                requires_grad)

        lo, hi = z_range
        p = LatticeParams()
        p.phi = [(u(batch, ny, nx, dt=real_dtype), u(batch, ny, nx, dt=real_dtype)) for _ in range(self.n_units)]
        p.wp = [u(batch, 2) for _ in range(self.n_units)]
        p.alpha = u(self.R * self.C, batch)
        zs = lo + (hi - lo) * torch.rand(2, self.nl, generator=gen, dtype=torch.float64)
        p.z1 = [torch.tensor(float(z), dtype=torch.float64, device=device, requires_grad=requires_grad)
                for z in zs[0]]
        p.z2 = [torch.tensor(float(z), dtype=torch.float64, device=device, requires_grad=requires_grad)
                for z in zs[1]]
        return p


def diagonal_units(R: int, C: int):
    """Unit mask with one building unit on the horizontal link entering each
    diagonal splitter (r, r): the discovery experiments place three units
    on the diagonal of the 3 x 3 grid."""
    mask = [False] * n_links(R, C)
    for r in range(min(R, C)):
        mask[h_link(R, C, r, r)] = True
    return mask


def transmittance(alpha):
    """[T, R] = [cos^2 alpha, sin^2 alpha] of splitter angles."""
    c = torch.cos(alpha.detach())
    return c * c, 1.0 - c * c


__all__ = ["Lattice", "LatticeParams", "diagonal_units", "n_links", "h_link", "v_link", "transmittance",
           "COMPONENTS"]
