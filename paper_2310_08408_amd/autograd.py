"""torch.autograd.Function wrappers: forward calls a libprop propagator,
backward calls its hand-written adjoint (the paper obtains these gradients
by reverse-mode autodiff; for a linear operator A the backward is A^H).

With torch's complex gradient convention (g = dL/dRe + i dL/dIm) the
gradient of an input x of y = A x is A^H g_y; for U = V exp(i phi) it is
dL/dphi = Im(g_U conj(U)) and g_V = g_U exp(-i phi).

RS and CZT also accept the distance z as a 0-d float64 tensor; when it
requires grad, backward returns dL/dz (rs_grad_z / czt_grad_z summed over
the batch, since one z is shared by all batch items).  The propagators take
z by value, so a device tensor is read back once per call; a caller that
already holds its value passes it as the optional last argument `zv`
(then z is not read).
"""
from __future__ import annotations

import torch

from . import (prop_sum_items, czt_adjoint, czt_grad_z, czt_propagate, prop_beam_splitter, prop_beam_splitter_adjoint,
               prop_density_loss, prop_modulate, prop_modulate_adjoint, prop_phase_grad, prop_phase_grad_sum,
               prop_scale_items, prop_softmin, prop_spot_loss, prop_waveplate,
               prop_waveplate_adjoint, prop_waveplate_batched, prop_waveplate_batched_adjoint, rs_adjoint,
               rs_adjoint_grad_z, rs_grad_z, rs_propagate, vczt_adjoint, vczt_propagate, vrs_adjoint, vrs_propagate)


def _zval(z):
    return float(z.detach()) if isinstance(z, torch.Tensor) else float(z)


class RS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, grid, wavelength, z, zv=None):
        u = u.contiguous()
        zv = _zval(z) if zv is None else float(zv)
        ctx.args = (grid, wavelength, zv)
        ctx.z_tensor = isinstance(z, torch.Tensor)
        ctx.z_shape = z.shape if ctx.z_tensor else None
        ctx.save_for_backward(u)
        return rs_propagate(u, grid, wavelength, zv)

    @staticmethod
    def backward(ctx, g):
        grid, wl, z = ctx.args
        (u,) = ctx.saved_tensors
        g = g.contiguous()
        gz = gu = None
        want_z = ctx.z_tensor and ctx.needs_input_grad[3]
        if want_z and ctx.needs_input_grad[0]:
            gu, dz = rs_adjoint_grad_z(g, u, grid, wl, z)
            gz = prop_sum_items(dz).reshape(ctx.z_shape)
        elif want_z:
            gz = prop_sum_items(rs_grad_z(u, g, grid, wl, z)).reshape(ctx.z_shape)
        elif ctx.needs_input_grad[0]:
            gu = rs_adjoint(g, grid, wl, z)
        return gu, None, None, gz, None


class CZT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, grid_in, window, wavelength, z, zv=None):
        u = u.contiguous()
        zv = _zval(z) if zv is None else float(zv)
        ctx.args = (grid_in, window, wavelength, zv)
        ctx.z_tensor = isinstance(z, torch.Tensor)
        ctx.z_shape = z.shape if ctx.z_tensor else None
        y = czt_propagate(u, grid_in, window, wavelength, zv)
        ctx.save_for_backward(u, y)
        return y

    @staticmethod
    def backward(ctx, g):
        gi, win, wl, z = ctx.args
        u, y = ctx.saved_tensors
        g = g.contiguous()
        gz = None
        if ctx.z_tensor and ctx.needs_input_grad[4]:
            gz = prop_sum_items(czt_grad_z(u, g, gi, win, wl, z, u_out=y)).reshape(ctx.z_shape)
        gu = czt_adjoint(g, gi, win, wl, z) if ctx.needs_input_grad[0] else None
        return gu, None, None, None, gz, None


class VRS(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ex, ey, grid, wavelength, z):
        ctx.args = (grid, wavelength, z)
        return vrs_propagate(ex.contiguous(), ey.contiguous(), grid, wavelength, z)

    @staticmethod
    def backward(ctx, gx, gy, gz):
        grid, wl, z = ctx.args
        ref = next(t for t in (gx, gy, gz) if t is not None)
        gx, gy, gz = (torch.zeros_like(ref) if t is None else t.contiguous() for t in (gx, gy, gz))
        gex, gey = vrs_adjoint(gx, gy, gz, grid, wl, z)
        return gex, gey, None, None, None


class VCZT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ex, ey, grid_in, window, wavelength, z, lens):
        ctx.args = (grid_in, window, wavelength, z, lens)
        return vczt_propagate(ex.contiguous(), ey.contiguous(), grid_in, window, wavelength, z, lens)

    @staticmethod
    def backward(ctx, gx, gy, gz):
        gi, win, wl, z, lens = ctx.args
        ref = next(t for t in (gx, gy, gz) if t is not None)
        gx, gy, gz = (torch.zeros_like(ref) if t is None else t.contiguous() for t in (gx, gy, gz))
        gex, gey = vczt_adjoint(gx, gy, gz, gi, win, wl, z, lens)
        return gex, gey, None, None, None, None, None


class Modulate(torch.autograd.Function):
    """SLM: U = V exp(i phi) (phi real, broadcast over the batch if shared)."""

    @staticmethod
    def forward(ctx, v, phase):
        v, phase = v.contiguous(), phase.contiguous()
        u = prop_modulate(v, phase)
        ctx.save_for_backward(u, phase)
        ctx.shared = phase.numel() != v.numel()
        return u

    @staticmethod
    def backward(ctx, g):
        u, phase = ctx.saved_tensors
        g = g.contiguous()
        g_v = prop_modulate_adjoint(g, phase) if ctx.needs_input_grad[0] else None
        g_phi = None
        if ctx.needs_input_grad[1]:
            if ctx.shared:
                g_phi = prop_phase_grad_sum(g, u).reshape(phase.shape)
            else:
                g_phi = prop_phase_grad(g, u)
        return g_v, g_phi


class WavePlate(torch.autograd.Function):
    """Jones retarder J(eta, theta) on (E_x, E_y); eta, theta are 0-d tensors."""

    @staticmethod
    def forward(ctx, ex, ey, eta, theta):
        ex, ey = ex.contiguous(), ey.contiguous()
        ctx.save_for_backward(ex, ey, eta, theta)
        return prop_waveplate(ex, ey, float(eta), float(theta))

    @staticmethod
    def backward(ctx, gx, gy):
        ex, ey, eta, theta = ctx.saved_tensors
        gx = torch.zeros_like(ex) if gx is None else gx.contiguous()
        gy = torch.zeros_like(ey) if gy is None else gy.contiguous()
        gex, gey, dp = prop_waveplate_adjoint(gx, gy, ex, ey, float(eta), float(theta))
        tot = prop_sum_items(dp)
        return gex, gey, tot[0].to(eta.dtype).reshape(eta.shape), tot[1].to(theta.dtype).reshape(theta.shape)


class WavePlates(torch.autograd.Function):
    """Wave plates with one (eta, theta) per batch item: params is a float64
    [batch, 2] device tensor."""

    @staticmethod
    def forward(ctx, ex, ey, params):
        ex, ey = ex.contiguous(), ey.contiguous()
        ctx.save_for_backward(ex, ey, params)
        return prop_waveplate_batched(ex, ey, params)

    @staticmethod
    def backward(ctx, gx, gy):
        ex, ey, params = ctx.saved_tensors
        gx = torch.zeros_like(ex) if gx is None else gx
        gy = torch.zeros_like(ey) if gy is None else gy
        gex, gey, dp = prop_waveplate_batched_adjoint(gx, gy, ex, ey, params, grad=ctx.needs_input_grad[2])
        return gex, gey, (dp.reshape(params.shape) if dp is not None else None)


class BeamSplitter(torch.autograd.Function):
    """Beam splitter with one mixing angle per batch item (alpha float64
    [batch]) on ncomp components per port:
    BeamSplitter.apply(ncomp, has_a, has_b, alpha, *a_planes, *b_planes)
    returns the ncomp planes of port c, then the ncomp planes of port d.
    A port flagged absent is dark and contributes no planes."""

    @staticmethod
    def forward(ctx, ncomp, has_a, has_b, alpha, *planes):
        a = list(planes[:ncomp]) if has_a else None
        b = list(planes[ncomp * int(has_a):]) if has_b else None
        c, d = prop_beam_splitter(a, b, alpha)
        ctx.ncomp, ctx.has_a, ctx.has_b = ncomp, has_a, has_b
        ctx.save_for_backward(alpha, *planes)
        return (*c, *d)

    @staticmethod
    def backward(ctx, *g):
        alpha, *planes = ctx.saved_tensors
        n, has_a, has_b = ctx.ncomp, ctx.has_a, ctx.has_b
        ref = next(t for t in list(g) + planes if t is not None)
        g = [torch.zeros_like(ref) if t is None else t for t in g]
        a = planes[:n] if has_a else None
        b = planes[n * int(has_a):] if has_b else None
        need = ctx.needs_input_grad
        want_a = has_a and any(need[4:4 + n])
        want_b = has_b and any(need[4 + n * int(has_a):])
        ga, gb, da = prop_beam_splitter_adjoint(g[:n], g[n:], a, b, alpha, (want_a, want_b), grad=need[3])
        outs = []
        if has_a:
            outs += list(ga) if ga is not None else [None] * n
        if has_b:
            outs += list(gb) if gb is not None else [None] * n
        return (None, None, None, da, *outs)


# ---------------------------------------------------------------------------
# Elements on stacked two-component fields S = [2, batch, ny, nx] (S[0] = E_x,
# S[1] = E_y).  A chain that keeps its fields stacked runs each scalar RS
# propagation once over 2 * batch planes (one launch set instead of two), and
# no element copies a component in or out of a stack: every output and every
# input gradient is written into the halves of one new tensor.


class ModulatePair(torch.autograd.Function):
    """SLMs on both components: E_x exp(i phi_x), E_y exp(i phi_y)."""

    @staticmethod
    def forward(ctx, s, phi_x, phi_y):
        s, phi_x, phi_y = s.contiguous(), phi_x.contiguous(), phi_y.contiguous()
        u = torch.empty_like(s)
        prop_modulate(s[0], phi_x, out=u[0])
        prop_modulate(s[1], phi_y, out=u[1])
        ctx.save_for_backward(u, phi_x, phi_y)
        return u

    @staticmethod
    def backward(ctx, g):
        u, phi_x, phi_y = ctx.saved_tensors
        g = g.contiguous()
        g_s = None
        if ctx.needs_input_grad[0]:
            g_s = torch.empty_like(g)
            prop_modulate_adjoint(g[0], phi_x, out=g_s[0])
            prop_modulate_adjoint(g[1], phi_y, out=g_s[1])
        g_phi = []
        for k, phi in enumerate((phi_x, phi_y)):
            if not ctx.needs_input_grad[1 + k]:
                g_phi.append(None)
            elif phi.numel() != u[k].numel():
                g_phi.append(prop_phase_grad_sum(g[k], u[k]).reshape(phi.shape))
            else:
                g_phi.append(prop_phase_grad(g[k], u[k]))
        return g_s, g_phi[0], g_phi[1]


class WavePlatesPair(torch.autograd.Function):
    """Wave plates with one (eta, theta) per batch item (params float64
    [batch, 2]) on a stacked field."""

    @staticmethod
    def forward(ctx, s, params):
        s = s.contiguous()
        o = torch.empty_like(s)
        prop_waveplate_batched(s[0], s[1], params, out=(o[0], o[1]))
        ctx.save_for_backward(s, params)
        return o

    @staticmethod
    def backward(ctx, g):
        s, params = ctx.saved_tensors
        g = g.contiguous()
        g_s = torch.empty_like(g)
        _, _, dp = prop_waveplate_batched_adjoint(g[0], g[1], s[0], s[1], params, grad=ctx.needs_input_grad[1],
                                                  out=(g_s[0], g_s[1]))
        return (g_s if ctx.needs_input_grad[0] else None), (dp.reshape(params.shape) if dp is not None else None)


class BeamSplitterPair(torch.autograd.Function):
    """Beam splitter with one mixing angle per batch item (alpha float64
    [batch]) on stacked ports: BeamSplitterPair.apply(alpha, S_a, S_b) ->
    (S_c, S_d); a dark input port is None (at most one)."""

    @staticmethod
    def forward(ctx, alpha, sa, sb):
        sa = sa.contiguous() if sa is not None else None
        sb = sb.contiguous() if sb is not None else None
        ref = sa if sa is not None else sb
        sc, sd = torch.empty_like(ref), torch.empty_like(ref)
        prop_beam_splitter([sa[0], sa[1]] if sa is not None else None, [sb[0], sb[1]] if sb is not None else None,
                           alpha, out=([sc[0], sc[1]], [sd[0], sd[1]]))
        ctx.save_for_backward(alpha, sa, sb)
        return sc, sd

    @staticmethod
    def backward(ctx, gc, gd):
        alpha, sa, sb = ctx.saved_tensors
        ref = next(t for t in (gc, gd, sa, sb) if t is not None)
        gc = torch.zeros_like(ref) if gc is None else gc.contiguous()
        gd = torch.zeros_like(ref) if gd is None else gd.contiguous()
        need = ctx.needs_input_grad
        want = (sa is not None and need[1], sb is not None and need[2])
        g_a = torch.empty_like(ref) if want[0] else None
        g_b = torch.empty_like(ref) if want[1] else None
        _, _, da = prop_beam_splitter_adjoint(
            [gc[0], gc[1]], [gd[0], gd[1]], [sa[0], sa[1]] if sa is not None else None,
            [sb[0], sb[1]] if sb is not None else None, alpha, want, grad=need[0],
            out=([g_a[0], g_a[1]] if want[0] else None, [g_b[0], g_b[1]] if want[1] else None))
        return da, g_a, g_b


class SpotLoss(torch.autograd.Function):
    """Per-field loss sigma^2/lambda^2 + w_fz F_z on ``window`` (shape [batch])."""

    @staticmethod
    def forward(ctx, ex, ey, ez, window, wavelength, w_fz):
        res, seeds = prop_spot_loss(ex.contiguous(), ey.contiguous(), None if ez is None else ez.contiguous(),
                                    window, wavelength, w_fz, seeds=True)
        ctx.seeds = seeds
        ctx.has_ez = ez is not None
        return res[:, 0].clone()

    @staticmethod
    def backward(ctx, g):
        # the seeds times the upstream gradient, into new planes (the kept
        # seeds serve further backward passes)
        planes = prop_scale_items([t for t in ctx.seeds if t is not None], g)
        return planes[0], planes[1], (planes[2] if ctx.has_ez else None), None, None, None


class DensityLoss(torch.autograd.Function):
    """Threshold-density loss Area / I_eps per batch item (float64 [batch]) of
    the intensity of the first `ncomp` fields, STED-modulated by the
    remaining fields (depletion beam) when there are any:
    DensityLoss.apply(ncomp, eps, beta, *fields)."""

    @staticmethod
    def forward(ctx, ncomp, eps, beta, *fields):
        comps, dep = list(fields[:ncomp]), list(fields[ncomp:])
        res, gs, gd = prop_density_loss(comps, eps, dep or None, beta, seeds=True)
        ctx.seeds = gs + gd
        return res[:, 0].clone()

    @staticmethod
    def backward(ctx, g):
        seeds = ctx.seeds
        out = []
        for k in range(0, len(seeds), 3):
            out += prop_scale_items(seeds[k:k + 3], g)
        return (None, None, None, *out)


class SoftMin(torch.autograd.Function):
    """Smooth minimum over the last axis of float64 losses [batch, ndet]."""

    @staticmethod
    def forward(ctx, losses, beta):
        val, w = prop_softmin(losses, beta)
        ctx.save_for_backward(w)
        return val

    @staticmethod
    def backward(ctx, g):
        (w,) = ctx.saved_tensors
        return g.reshape(-1, 1) * w, None

