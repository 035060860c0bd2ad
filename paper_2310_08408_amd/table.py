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
wave plates (J(eta, theta)^H) from C, so no propagation is recomputed; the
linear propagators need no saved state at all.  Up to wave plate 1 both
polarisation components carry the same scalar field, so SLM1, RS and SLM2
run once per set, and wave plate 1's adjoint folds its two component
gradients into the one field's.  The wave-plate parameters of all sets are
one device array, so every element is one launch for the whole batch.
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
        """phi1, phi2: [B, ny, nx] real; wp1, wp2: per set (eta, theta) pairs
        (sequences of B pairs, or float64 [B, 2] tensors).  Returns the
        per-set loss [B] (float64) and keeps the checkpoints."""
        g, wl = self.grid, self.wl
        dev = phi1.device
        w1 = torch.as_tensor(wp1, dtype=torch.float64).reshape(self.batch, 2).to(dev)
        w2 = torch.as_tensor(wp2, dtype=torch.float64).reshape(self.batch, 2).to(dev)
        u1 = lp.prop_modulate(self.v, phi1)                       # checkpoint 1 (enters RS)
        s = lp.rs_propagate(u1, g, wl, self.z)
        a = lp.prop_modulate(s, phi2)
        bx, by = lp.prop_waveplate_batched(a, a, w1)
        cx, cy = lp.prop_waveplate_batched(bx, by, w2)            # checkpoint 2 (enters VCZT)
        ex, ey, ez = lp.vczt_propagate(cx, cy, g, self.window, wl, lens=self.lens)
        res, seeds = lp.prop_spot_loss(ex, ey, ez, self.window, wl, self.w_fz, seeds=True)
        self.saved = (u1, cx, cy, phi1, phi2, w1, w2, seeds)
        return res[:, 0].clone()

    def backward(self):
        """Gradients of sum(loss): (g_phi1 [B,ny,nx], g_phi2, g_wp1 [B,2], g_wp2 [B,2])."""
        u1, cx, cy, phi1, phi2, w1, w2, seeds = self.saved
        g, wl = self.grid, self.wl
        gcx, gcy = lp.vczt_adjoint(*seeds, g, self.window, wl, lens=self.lens)
        # wave plate 2: its input from the checkpoint through J2^H
        bx, by, _ = lp.prop_waveplate_batched_adjoint(cx, cy, None, None, w2, grad=False)
        gbx, gby, g_wp2 = lp.prop_waveplate_batched_adjoint(gcx, gcy, bx, by, w2)
        # wave plate 1 was fed (A, A): A = (J1^H B)_x, and its adjoint sums the
        # two component gradients into g_A
        a, _, _ = lp.prop_waveplate_batched_adjoint(bx, by, None, None, w1, grad=False)
        ga, _, g_wp1 = lp.prop_waveplate_batched_adjoint(gbx, gby, a, a, w1, shared_input=True)
        g_phi2 = lp.prop_phase_grad(ga, a)
        gs = lp.prop_modulate_adjoint(ga, phi2)
        gu1 = lp.rs_adjoint(gs, g, wl, self.z)
        g_phi1 = lp.prop_phase_grad(gu1, u1)
        return g_phi1, g_phi2, g_wp1, g_wp2
