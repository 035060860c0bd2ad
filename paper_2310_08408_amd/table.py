"""Checkpointed virtual optical table: forward and hand-written backward.

Chain per parameter set (paper: Results, STED / sharp-focus setups built
from SLMs, wave plates and a high-NA objective; Methods, SLM and variable
retarders):

    V (Gaussian, linear 45 deg polarisation: E_x = E_y = V / sqrt 2)
    -> SLM1 (phase phi1) -> RS over z -> SLM2 (phase phi2)
    -> wave plate 1 (eta1, theta1) -> wave plate 2 (eta2, theta2)
    -> high-NA objective (VCZT focusing) -> loss sigma^2/lambda^2 + w_fz F_z.

Checkpointing: only the fields entering the two propagations are kept
(U1 = SLM1 output, scalar; C = wave-plate-2 output, two components).  The
backward recovers the elementwise intermediates by inverting the unitary
wave plates (J(eta, theta)^H = J(-eta, theta)) from C, so no propagation is
recomputed; the linear propagators need no saved state at all.  Up to
wave plate 1 both polarisation components carry the same scalar field, so
SLM1, RS and SLM2 run once per set.
"""
from __future__ import annotations

import math

import torch

import paper_2310_08408_amd as lp


class OpticalTable:
    def __init__(self, grid, window, wavelength, w0, z, na, f, batch, dtype=torch.complex64, w_fz=1.0):
        self.grid, self.window, self.wl, self.z = grid, window, wavelength, z
        self.lens = (na, f)
        self.batch, self.dtype, self.w_fz = batch, dtype, w_fz
        self.rdt = torch.float32 if dtype == torch.complex64 else torch.float64
        self.v = lp.prop_source_gaussian(grid, w0, wavelength, amplitude=1.0 / math.sqrt(2.0), batch=batch,
                                         dtype=dtype)

    def forward(self, phi1, phi2, wp1, wp2):
        """phi1, phi2: [B, ny, nx] real; wp1, wp2: per set (eta, theta) pairs.
        Returns the per-set loss [B] (float64) and keeps the checkpoints."""
        g, wl = self.grid, self.wl
        u1 = lp.prop_modulate(self.v, phi1)                       # checkpoint 1 (enters RS)
        s = lp.rs_propagate(u1, g, wl, self.z)
        a = lp.prop_modulate(s, phi2)
        cx, cy = torch.empty_like(a), torch.empty_like(a)
        for b in range(self.batch):
            bx, by = lp.prop_waveplate(a[b:b + 1], a[b:b + 1], *wp1[b])
            ox, oy = lp.prop_waveplate(bx, by, *wp2[b])
            cx[b:b + 1].copy_(ox)
            cy[b:b + 1].copy_(oy)
        ex, ey, ez = lp.vczt_propagate(cx, cy, g, self.window, wl, lens=self.lens)
        res, seeds = lp.prop_spot_loss(ex, ey, ez, self.window, wl, self.w_fz, seeds=True)
        self.saved = (u1, cx, cy, phi1, phi2, list(wp1), list(wp2), seeds)
        return res[:, 0].clone()

    def backward(self):
        """Gradients of sum(loss): (g_phi1 [B,ny,nx], g_phi2, g_wp1 [B,2], g_wp2 [B,2])."""
        u1, cx, cy, phi1, phi2, wp1, wp2, seeds = self.saved
        g, wl = self.grid, self.wl
        gcx, gcy = lp.vczt_adjoint(*seeds, g, self.window, wl, lens=self.lens)
        ga = torch.empty_like(cx)
        a = torch.empty_like(cx)
        g_wp1 = torch.empty((self.batch, 2), dtype=torch.float64, device=cx.device)
        g_wp2 = torch.empty_like(g_wp1)
        for b in range(self.batch):
            sl = slice(b, b + 1)
            e2, t2 = wp2[b]
            e1, t1 = wp1[b]
            # wave plate 2: its input from the checkpoint through J2^H = J(-eta2, theta2)
            bx, by = lp.prop_waveplate(cx[sl], cy[sl], -e2, t2)
            gbx, gby, d2 = lp.prop_waveplate_adjoint(gcx[sl], gcy[sl], bx, by, e2, t2)
            # wave plate 1: its input is (A, A) = J1^H (B)
            ax, ay = lp.prop_waveplate(bx, by, -e1, t1)
            gax, gay, d1 = lp.prop_waveplate_adjoint(gbx, gby, ax, ay, e1, t1)
            ga[sl].copy_(gax + gay)        # both components came from the same scalar A
            a[sl].copy_(ax)
            g_wp1[b] = d1[0]
            g_wp2[b] = d2[0]
        g_phi2 = lp.prop_phase_grad(ga, a)
        gs = lp.prop_modulate(ga, -phi2)
        gu1 = lp.rs_adjoint(gs, g, wl, self.z)
        g_phi1 = lp.prop_phase_grad(gu1, u1)
        return g_phi1, g_phi2, g_wp1, g_wp2
