"""FP64 CPU oracle for multi-element optical tables -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; nothing here imports the library.

The paper's large-scale ansatz (Results, Fig. "General virtual optical setup
for large-scale discovery"; Methods, "The large-scale search space") joins
building units -- a super-SLM and a wave plate a distance z1 apart -- through
free propagation over z2 and beam splitters.  Its 3x3 instance has six
sources, nine beam splitters, 24 super-SLMs, 24 wave plates and six
high-NA detectors.  The paper gives the element counts and the ratios it
found, but neither the beam-splitter matrix nor the wiring.  Readings:

L1 beam splitter: lossless, symmetric and polarisation independent with
   mixing angle alpha (transmittance T = cos^2 alpha, reflectance
   R = sin^2 alpha; the paper reports [T, R] pairs in [0, 1]):
       c = cos(alpha) a + i sin(alpha) b,   d = i sin(alpha) a + cos(alpha) b
   (a: port entering from the left, b: from the top; c leaves to the
   right, d downwards).  The angle parametrisation keeps dL/dalpha finite
   at T = 0 and T = 1.
L2 wiring: an R x C lattice of beam splitters.  Source r (r < R) enters row
   r from the left, source R + c enters column c from the top; detector r
   sits at the right end of row r, detector R + c at the bottom of column
   c.  A link -- source to splitter, splitter to splitter, splitter to
   detector -- may hold a building unit: super-SLM (phase phi_x on E_x,
   phi_y on E_y), propagation over z1, wave plate (eta, theta).  Every
   link then propagates over its own distance z2 (z2 = 0: none).  With a
   unit on each of the 24 links of R = C = 3 the element counts are those of
   the large-scale setup in Methods; the discovery experiments put three
   units on the diagonal of the same grid.
L3 propagation between elements: the transverse part of vectorial RS,
   which is the scalar RS integral applied to E_x and to E_y.  No element
   between propagations acts on E_z, and vectorial RS rebuilds E_z from the
   transverse field of its input plane, so E_z is formed only at the
   detectors, whose high-NA objective (Richards-Wolf focusing onto the
   detector window) yields (E_x, E_y, E_z).
L4 detector loss: the threshold-density loss of the chosen components
   ('ez': |E_z|^2, 'radial': |E_x|^2 + |E_y|^2, 'total': all three) per
   detector, STED-modulated by a second beam (depletion) through the same
   lattice at its own wavelength when one is given; the objective is the
   soft minimum over the detectors (Methods, exploration of optical
   topologies).
L5 beams of different wavelengths do not interfere: each runs through the
   lattice on its own, with the same element parameters.

Link numbering: horizontal link (r, j), j = 0..C, has index r (C + 1) + j;
vertical link (i, c), i = 0..R, has index R (C + 1) + c (R + 1) + i.
"""
from __future__ import annotations

import math

import numpy as np

from .optics import (C128, density_loss_fields, modulate, phase_grad, rs_adjoint, rs_grad_z, rs_propagate,
                     softmin, vczt_focus, vczt_focus_adjoint, waveplate, waveplate_adjoint)

COMPONENTS = {"ez": (2,), "radial": (0, 1), "total": (0, 1, 2)}


# --------------------------------------------------------------------------
# Beam splitter (L1)
# --------------------------------------------------------------------------

def beam_splitter(a, b, alpha: float):
    """Outputs (c, d) of the splitter for input ports a, b (sequences of
    field components; None = dark port)."""
    ca, sa = math.cos(alpha), math.sin(alpha)
    a, b = _ports(a, b)
    c = [ca * x + 1j * sa * y for x, y in zip(a, b)]
    d = [1j * sa * x + ca * y for x, y in zip(a, b)]
    return c, d


def beam_splitter_adjoint(gc, gd, a, b, alpha: float):
    """(g_a, g_b, dL/dalpha) for (c, d) = beam_splitter(a, b, alpha): the
    input gradients apply the conjugate transpose [[cos, -i sin], [-i sin,
    cos]]; dL/dalpha = Re sum conj(g_c) dc/dalpha + conj(g_d) dd/dalpha
    (gradient convention g = dL/dRe + i dL/dIm)."""
    ca, sa = math.cos(alpha), math.sin(alpha)
    a, b = _ports(a, b)
    gc = [np.asarray(g, dtype=C128) for g in gc]
    gd = [np.asarray(g, dtype=C128) for g in gd]
    ga = [ca * x - 1j * sa * y for x, y in zip(gc, gd)]
    gb = [-1j * sa * x + ca * y for x, y in zip(gc, gd)]
    dal = 0.0
    for x, y, p, q in zip(a, b, gc, gd):
        dc = -sa * x + 1j * ca * y
        dd = 1j * ca * x - sa * y
        dal += float(np.sum(np.real(np.conj(p) * dc + np.conj(q) * dd)))
    return ga, gb, dal


def _ports(a, b):
    ref = a if a is not None else b
    ref = [np.asarray(x, dtype=C128) for x in ref]
    z = [np.zeros_like(x) for x in ref]
    a = z if a is None else [np.asarray(x, dtype=C128) for x in a]
    b = z if b is None else [np.asarray(x, dtype=C128) for x in b]
    return a, b


# --------------------------------------------------------------------------
# Lattice wiring (L2)
# --------------------------------------------------------------------------

def n_links(R: int, C: int) -> int:
    return R * (C + 1) + C * (R + 1)


def h_link(R: int, C: int, r: int, j: int) -> int:
    return r * (C + 1) + j


def v_link(R: int, C: int, i: int, c: int) -> int:
    return R * (C + 1) + c * (R + 1) + i


def run_lattice(R: int, C: int, sources, alpha, link_fwd):
    """Forward wiring of one beam.  sources: R + C entries, each a list of
    transverse components or None; alpha[r][c]; link_fwd(l, field) -> field.
    Returns (detector fields [R + C], splitter inputs {(r, c): (a, b)})."""
    ref = next(s for s in sources if s is not None)
    dark = [np.zeros_like(np.asarray(x, dtype=C128)) for x in ref]
    src = [dark if s is None else [np.asarray(x, dtype=C128) for x in s] for s in sources]
    h_in = {(r, 0): src[r] for r in range(R)}
    v_in = {(0, c): src[R + c] for c in range(C)}
    bs_in = {}
    for r in range(R):
        for c in range(C):
            a = link_fwd(h_link(R, C, r, c), h_in[(r, c)])
            b = link_fwd(v_link(R, C, r, c), v_in[(r, c)])
            bs_in[(r, c)] = (a, b)
            h_in[(r, c + 1)], v_in[(r + 1, c)] = beam_splitter(a, b, alpha[r][c])
    det = [link_fwd(h_link(R, C, r, C), h_in[(r, C)]) for r in range(R)]
    det += [link_fwd(v_link(R, C, R, c), v_in[(R, c)]) for c in range(C)]
    return det, bs_in


def run_lattice_adjoint(R: int, C: int, g_det, bs_in, alpha, link_bwd):
    """Reverse wiring of one beam: g_det[R + C] detector-field gradients;
    link_bwd(l, g_out) -> g_in (and records the link's parameter gradients).
    Returns dL/dalpha[R][C]."""
    g_h = {(r, C): link_bwd(h_link(R, C, r, C), g_det[r]) for r in range(R)}
    g_v = {(R, c): link_bwd(v_link(R, C, R, c), g_det[R + c]) for c in range(C)}
    dal = np.zeros((R, C))
    for r in reversed(range(R)):
        for c in reversed(range(C)):
            a, b = bs_in[(r, c)]
            ga, gb, dal[r, c] = beam_splitter_adjoint(g_h[(r, c + 1)], g_v[(r + 1, c)], a, b, alpha[r][c])
            g_h[(r, c)] = link_bwd(h_link(R, C, r, c), ga)
            g_v[(r, c)] = link_bwd(v_link(R, C, r, c), gb)
    return dal


# --------------------------------------------------------------------------
# Building unit and the full objective (L2-L5)
# --------------------------------------------------------------------------

def lattice_objective(R: int, C: int, g, win, beams, params, na: float, f: float, eps: float,
                      comps: str = "ez", beta_sted: float = 1.0, beta_soft: float = 10.0):
    """One parameter set of the lattice and its gradients.

    g, win: grids of the links and of the detector windows.
    beams: list of 1 or 2 dicts {"wavelength", "sources"} (sources: R + C
      transverse fields [ex, ey] or None); a second beam is the depletion
      beam of the STED modulation (L4, L5).
    params: dict with
      "unit"  [nlinks] bool, which links hold a building unit,
      "phi"   [nunits, 2, ny, nx] super-SLM phases (E_x, E_y) of the units
              in link order,
      "wp"    [nunits, 2] wave plate (eta, theta),
      "alpha" [R, C] splitter angles,
      "z1"    [nlinks] super-SLM to wave plate distance (units only),
      "z2"    [nlinks] propagation distance of every link (0: none).
    Returns (objective, per-detector losses, grads {"phi", "wp", "alpha",
    "z1", "z2"}).
    """
    nl = n_links(R, C)
    unit = [bool(x) for x in params["unit"]]
    uidx = list(np.cumsum(unit) - 1)
    phi, wp, alpha = params["phi"], params["wp"], params["alpha"]
    z1, z2 = params["z1"], params["z2"]
    sel = COMPONENTS[comps]
    runs = []
    for beam in beams:
        wl = beam["wavelength"]
        saved = {}

        def link_fwd(l, x, wl=wl, saved=saved):
            u = p = None
            w = x
            if unit[l]:
                k = uidx[l]
                u = [modulate(x[0], phi[k][0]), modulate(x[1], phi[k][1])]
                p = [rs_propagate(u[0], g, wl, z1[l]), rs_propagate(u[1], g, wl, z1[l])]
                w = list(waveplate(p[0], p[1], wp[k][0], wp[k][1]))
            o = [rs_propagate(w[0], g, wl, z2[l]), rs_propagate(w[1], g, wl, z2[l])] if z2[l] > 0 else w
            saved[l] = (u, p, w)
            return o

        det, bs_in = run_lattice(R, C, beam["sources"], alpha, link_fwd)
        fields = [vczt_focus(d[0], d[1], g, win, wl, na, f) for d in det]
        runs.append((wl, saved, bs_in, fields))
    ndet = R + C
    losses, seeds = np.zeros(ndet), []
    for k in range(ndet):
        ex_f = [runs[0][3][k][c] for c in sel]
        dep_f = [runs[1][3][k][c] for c in sel] if len(runs) > 1 else None
        loss, _, _, _, s_ex, s_dep = density_loss_fields(ex_f, eps, dep_f, beta_sted)
        losses[k] = loss
        seeds.append((s_ex, s_dep))
    obj, wts = softmin(losses, beta_soft)

    grads = {"phi": np.zeros(np.shape(phi)), "wp": np.zeros(np.shape(wp)), "alpha": np.zeros((R, C)),
             "z1": np.zeros(nl), "z2": np.zeros(nl)}
    for bi, (wl, saved, bs_in, fields) in enumerate(runs):
        g_det = []
        for k in range(ndet):
            s = seeds[k][bi]
            gfull = [np.zeros_like(fields[k][0]) for _ in range(3)]
            for c, sc in zip(sel, s):
                gfull[c] = wts[k] * sc
            g_det.append(list(vczt_focus_adjoint(gfull[0], gfull[1], gfull[2], g, win, wl, na, f)))

        def link_bwd(l, go, wl=wl, saved=saved):
            u, p, w = saved[l]
            gw = go
            if z2[l] > 0:
                gw = [rs_adjoint(go[0], g, wl, z2[l]), rs_adjoint(go[1], g, wl, z2[l])]
                grads["z2"][l] += rs_grad_z(w[0], go[0], g, wl, z2[l]) + rs_grad_z(w[1], go[1], g, wl, z2[l])
            if not unit[l]:
                return gw
            k = uidx[l]
            gpx, gpy, de, dt = waveplate_adjoint(gw[0], gw[1], p[0], p[1], wp[k][0], wp[k][1])
            grads["wp"][k] += (de, dt)
            grads["z1"][l] += rs_grad_z(u[0], gpx, g, wl, z1[l]) + rs_grad_z(u[1], gpy, g, wl, z1[l])
            gu = [rs_adjoint(gpx, g, wl, z1[l]), rs_adjoint(gpy, g, wl, z1[l])]
            for c in range(2):
                grads["phi"][k, c] += phase_grad(gu[c], u[c])
            return [gu[c] * np.exp(-1j * np.asarray(phi[k][c], dtype=np.float64)) for c in range(2)]

        grads["alpha"] += run_lattice_adjoint(R, C, g_det, bs_in, alpha, link_bwd)
    return obj, losses, grads


def path_sum(R: int, C: int, alpha, link_phase, src: int, det: int) -> complex:
    """Amplitude from source ``src`` to detector ``det`` of a lattice whose
    links multiply by exp(i link_phase[l]) (scalar light), as an explicit sum
    over all monotone paths: a splitter contributes cos(alpha) where the
    path keeps its direction and i sin(alpha) where it turns (L1, L2)."""
    total = 0j

    def walk(r, c, heading, amp):
        # standing on the input port of splitter (r, c) (or past the lattice)
        nonlocal total
        if heading == "h" and c == C:
            if det == r:
                total += amp * np.exp(1j * link_phase[h_link(R, C, r, C)])
            return
        if heading == "v" and r == R:
            if det == R + c:
                total += amp * np.exp(1j * link_phase[v_link(R, C, R, c)])
            return
        l = h_link(R, C, r, c) if heading == "h" else v_link(R, C, r, c)
        amp = amp * np.exp(1j * link_phase[l])
        t, s = math.cos(alpha[r][c]), 1j * math.sin(alpha[r][c])
        if heading == "h":
            walk(r, c + 1, "h", amp * t)
            walk(r + 1, c, "v", amp * s)
        else:
            walk(r + 1, c, "v", amp * t)
            walk(r, c + 1, "h", amp * s)

    if src < R:
        walk(src, 0, "h", 1.0 + 0j)
    else:
        walk(0, src - R, "v", 1.0 + 0j)
    return complex(total)
