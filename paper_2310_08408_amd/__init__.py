"""libprop Python binding: RS / CZT / VRS / VCZT light propagation and exact
adjoints on one MI355X, behind the C ABI of include/libprop.h.

Every function here marshals torch tensors (device memory, current stream)
into one libprop call; all arithmetic runs in the library's HIP kernels.
Fields are complex64 or complex128 CUDA(HIP) tensors shaped [..., ny, nx];
leading dimensions form the batch.  Real parameter tensors (phases) use the
matching real dtype.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

from . import _lib
from ._lib import PropError, PropWarning  # noqa: F401

__all__ = [
    "rs_propagate", "rs_adjoint", "czt_propagate", "czt_adjoint", "vrs_propagate", "vrs_adjoint",
    "vczt_propagate", "vczt_adjoint", "rs_grad_z", "rs_adjoint_grad_z", "czt_grad_z", "rs_adjoint_phase_grad",
    "czt_adjoint_phase_grad",
    "prop_source_gaussian", "prop_source_radial", "prop_modulate",
    "prop_phase_grad", "prop_waveplate", "prop_waveplate_adjoint", "prop_spot_loss", "prop_density_loss",
    "prop_softmin", "prop_adam_step", "Adam", "prop_track_best", "prop_sum_items", "StopRule", "prop_sampling_check",
    "prop_fft_length", "prop_cache_clear", "prop_trace_enable", "prop_trace_read", "prop_trace_only", "prop_autotune_report",
    "PropError", "PropWarning", "library", "Plan", "Setup", "PROP_OP_RS", "PROP_OP_CZT", "PROP_OP_VRS",
    "PROP_OP_VCZT", "PROP_OP_RS_CZT", "PROP_PLAN_GRAPH", "prop_tune_cache_path", "prop_tune_cache_rejected", "PROP_PLAN_AUTOTUNE", "PROP_PLAN_FAULT_NOMEM", "prop_cache_set_limit",
    "prop_cache_info",
]


def library():
    return _lib.load()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return _lib.PROP_C64
    if t.dtype == torch.complex128:
        return _lib.PROP_C128
    raise TypeError(f"expected complex64/complex128, got {t.dtype}")


def _real_dtype(t: torch.Tensor):
    return torch.float32 if t.dtype == torch.complex64 else torch.float64


def _dev(t: torch.Tensor, name: str = "tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: libprop operates on GPU tensors")
    if not t.is_contiguous():
        raise ValueError(f"{name}: libprop needs contiguous tensors")
    return t


def _arg(t, name, ref, grid=None, items=None, real=False, dtype=None):
    """Check one tensor argument against the call's reference tensor before
    its pointer reaches the library: a contiguous GPU tensor on ref's device,
    of ref's dtype (its real counterpart with real=True, or `dtype`), and --
    with `grid` -- shaped [..., ny, nx] with `items` planes (every pointer
    the library receives addresses items * ny * nx elements)."""
    _dev(t, name)
    if t.device != ref.device:
        raise ValueError(f"{name}: on {t.device}, the call's fields are on {ref.device}")
    want = dtype if dtype is not None else (_real_dtype(ref) if real else ref.dtype)
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
    if grid is not None:
        ny, nx = int(grid.ny), int(grid.nx)
        if t.dim() < 2 or t.shape[-1] != nx or t.shape[-2] != ny:
            raise ValueError(f"{name}: shape {tuple(t.shape)} does not end in (ny, nx) = ({ny}, {nx})")
        if items is not None and t.numel() != items * ny * nx:
            raise ValueError(f"{name}: {t.numel() // (ny * nx)} planes, expected {items}")
    return t


class _Plane:
    """(ny, nx) of a reference tensor's last two dimensions, as a grid."""

    def __init__(self, t):
        if t.dim() < 2:
            raise ValueError(f"expected [..., ny, nx], got shape {tuple(t.shape)}")
        self.ny, self.nx = int(t.shape[-2]), int(t.shape[-1])


def _field(t, name="u"):
    """The reference field of a call: a contiguous complex GPU tensor."""
    _dev(t, name)
    _dtype_code(t)
    return t


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _batch(t: torch.Tensor, g) -> int:
    n = int(g.nx) * int(g.ny)
    if t.dim() < 2 or t.shape[-1] != int(g.nx) or t.shape[-2] != int(g.ny):
        raise ValueError(f"tensor shape {tuple(t.shape)} does not end in (ny, nx) = ({g.ny}, {g.nx})")
    return t.numel() // n


def _like(t: torch.Tensor, g, out):
    shape = tuple(t.shape[:-2]) + (int(g.ny), int(g.nx))
    if out is None:
        return torch.empty(shape, dtype=t.dtype, device=t.device)
    _arg(out, "out", t)
    if tuple(out.shape) != shape:
        raise ValueError(f"out: shape {tuple(out.shape)}, expected {shape}")
    return out


# ------------------------------------------------------------------ RS / CZT --

def rs_propagate(u, grid, wavelength, z, out=None):
    """Scalar RS over z onto the input grid (see include/libprop.h)."""
    lib = library()
    _field(u)
    out = _like(u, grid, out)
    with torch.cuda.device(u.device):
        st = lib.rs_propagate(_dtype_code(u), _ptr(u), _ptr(out), ctypes.byref(_lib.grid(grid)), float(wavelength),
                              float(z), _batch(u, grid), _stream(u))
    _lib.check("rs_propagate", st)
    return out


def rs_adjoint(g_out, grid, wavelength, z, out=None):
    lib = library()
    _field(g_out, "g_out")
    out = _like(g_out, grid, out)
    with torch.cuda.device(g_out.device):
        st = lib.rs_adjoint(_dtype_code(g_out), _ptr(g_out), _ptr(out), ctypes.byref(_lib.grid(grid)),
                            float(wavelength), float(z), _batch(g_out, grid), _stream(g_out))
    _lib.check("rs_adjoint", st)
    return out


def czt_propagate(u, grid_in, window, wavelength, z, out=None):
    """Fresnel/CZT propagation over z onto ``window``."""
    lib = library()
    _field(u)
    b = _batch(u, grid_in)
    out = _like(u, window, out)
    with torch.cuda.device(u.device):
        st = lib.czt_propagate(_dtype_code(u), _ptr(u), _ptr(out), ctypes.byref(_lib.grid(grid_in)),
                               ctypes.byref(_lib.grid(window)), float(wavelength), float(z), b, _stream(u))
    _lib.check("czt_propagate", st)
    return out


def czt_adjoint(g_out, grid_in, window, wavelength, z, out=None):
    lib = library()
    _field(g_out, "g_out")
    b = _batch(g_out, window)
    out = _like(g_out, grid_in, out)
    with torch.cuda.device(g_out.device):
        st = lib.czt_adjoint(_dtype_code(g_out), _ptr(g_out), _ptr(out), ctypes.byref(_lib.grid(grid_in)),
                             ctypes.byref(_lib.grid(window)), float(wavelength), float(z), b, _stream(g_out))
    _lib.check("czt_adjoint", st)
    return out


# --------------------------------------------------------------- VRS / VCZT --

def _phase_grad_out(u, grid, grad, g_u):
    b = _batch(u, grid)
    if grad is None:
        grad = torch.empty(u.shape, dtype=_real_dtype(u), device=u.device)
    _arg(grad, "grad", u, grid, b, real=True)
    gu = torch.empty_like(u) if g_u is True else g_u
    gu = gu if gu is not None and gu is not False else None
    if gu is not None:
        _arg(gu, "g_u", u, grid, b)
    return grad, gu


def rs_adjoint_phase_grad(g_out, u, grid, wavelength, z, grad=None, accumulate=False, g_u=None):
    """RS adjoint fused with the SLM phase gradient: grad (+)= Im(g_U conj u),
    g_U = rs_adjoint(g_out).  g_u=True also returns g_U (or pass a tensor).
    Returns (grad, g_U or None)."""
    lib = library()
    _field(u)
    b = _batch(u, grid)
    _arg(g_out, "g_out", u, grid, b)
    grad, gu = _phase_grad_out(u, grid, grad, g_u)
    with torch.cuda.device(u.device):
        st = lib.rs_adjoint_phase_grad(_dtype_code(u), _ptr(g_out), _ptr(u), _ptr(gu), _ptr(grad),
                                       1 if accumulate else 0, ctypes.byref(_lib.grid(grid)), float(wavelength),
                                       float(z), b, _stream(u))
    _lib.check("rs_adjoint_phase_grad", st)
    return grad, gu


def czt_adjoint_phase_grad(g_out, u, grid_in, window, wavelength, z, grad=None, accumulate=False, g_u=None):
    """CZT adjoint fused with the SLM phase gradient (see rs_adjoint_phase_grad)."""
    lib = library()
    _field(u)
    b = _batch(u, grid_in)
    _arg(g_out, "g_out", u, window, b)
    grad, gu = _phase_grad_out(u, grid_in, grad, g_u)
    with torch.cuda.device(u.device):
        st = lib.czt_adjoint_phase_grad(_dtype_code(u), _ptr(g_out), _ptr(u), _ptr(gu), _ptr(grad),
                                        1 if accumulate else 0, ctypes.byref(_lib.grid(grid_in)),
                                        ctypes.byref(_lib.grid(window)), float(wavelength), float(z), b, _stream(u))
    _lib.check("czt_adjoint_phase_grad", st)
    return grad, gu


def rs_grad_z(u, g_out, grid, wavelength, z):
    """dL/dz per batch item (float64 tensor [batch]) for the RS propagation of
    u with output gradient seed g_out."""
    lib = library()
    _field(u)
    b = _batch(u, grid)
    _arg(g_out, "g_out", u, grid, b)
    dz = torch.empty((b,), dtype=torch.float64, device=u.device)
    with torch.cuda.device(u.device):
        st = lib.rs_grad_z(_dtype_code(u), _ptr(u), _ptr(g_out), _ptr(dz), ctypes.byref(_lib.grid(grid)),
                           float(wavelength), float(z), b, _stream(u))
    _lib.check("rs_grad_z", st)
    return dz


def rs_adjoint_grad_z(g_out, u, grid, wavelength, z, out=None):
    """rs_adjoint(g_out) and rs_grad_z(u, g_out) of one RS step in one call
    (the distance gradient shares the adjoint's first pass).  Returns
    (g_u, dz): g_u like u, dz float64 [batch]."""
    lib = library()
    _field(u)
    b = _batch(u, grid)
    _arg(g_out, "g_out", u, grid, b)
    out = _like(u, grid, out)
    dz = torch.empty((b,), dtype=torch.float64, device=u.device)
    with torch.cuda.device(u.device):
        st = lib.rs_adjoint_grad_z(_dtype_code(u), _ptr(g_out), _ptr(u), _ptr(out), _ptr(dz),
                                   ctypes.byref(_lib.grid(grid)), float(wavelength), float(z), b, _stream(u))
    _lib.check("rs_adjoint_grad_z", st)
    return out, dz


def czt_grad_z(u, g_out, grid_in, window, wavelength, z, u_out=None):
    """dL/dz per batch item for the CZT propagation of u onto `window` with
    output gradient seed g_out; u_out = czt_propagate(u, ...) if available."""
    lib = library()
    _field(u)
    b = _batch(u, grid_in)
    _arg(g_out, "g_out", u, window, b)
    if u_out is not None:
        _arg(u_out, "u_out", u, window, b)
    dz = torch.empty((b,), dtype=torch.float64, device=u.device)
    with torch.cuda.device(u.device):
        st = lib.czt_grad_z(_dtype_code(u), _ptr(u), _ptr(u_out), _ptr(g_out), _ptr(dz),
                            ctypes.byref(_lib.grid(grid_in)), ctypes.byref(_lib.grid(window)), float(wavelength),
                            float(z), b, _stream(u))
    _lib.check("czt_grad_z", st)
    return dz


def vrs_propagate(ex, ey, grid, wavelength, z):
    lib = library()
    _field(ex, "ex")
    b = _batch(ex, grid)
    _arg(ey, "ey", ex, grid, b)
    ox, oy, oz = (torch.empty_like(ex) for _ in range(3))
    with torch.cuda.device(ex.device):
        st = lib.vrs_propagate(_dtype_code(ex), _ptr(ex), _ptr(ey), _ptr(ox), _ptr(oy), _ptr(oz),
                               ctypes.byref(_lib.grid(grid)), float(wavelength), float(z), b, _stream(ex))
    _lib.check("vrs_propagate", st)
    return ox, oy, oz


def vrs_adjoint(gx, gy, gz, grid, wavelength, z):
    lib = library()
    _field(gx, "gx")
    b = _batch(gx, grid)
    _arg(gy, "gy", gx, grid, b), _arg(gz, "gz", gx, grid, b)
    gex, gey = torch.empty_like(gx), torch.empty_like(gx)
    with torch.cuda.device(gx.device):
        st = lib.vrs_adjoint(_dtype_code(gx), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gex), _ptr(gey),
                             ctypes.byref(_lib.grid(grid)), float(wavelength), float(z), b, _stream(gx))
    _lib.check("vrs_adjoint", st)
    return gex, gey


def _lens(lens):
    if lens is None:
        return None
    na, f = (lens.na, lens.f) if hasattr(lens, "na") else lens
    return ctypes.byref(_lib.prop_lens(float(na), float(f)))


def vczt_propagate(ex, ey, grid_in, window, wavelength, z=0.0, lens=None):
    """Vectorial CZT; ``lens=(na, f)`` selects the focusing (objective) mode."""
    lib = library()
    _field(ex, "ex")
    b = _batch(ex, grid_in)
    _arg(ey, "ey", ex, grid_in, b)
    ox, oy, oz = (_like(ex, window, None) for _ in range(3))
    with torch.cuda.device(ex.device):
        st = lib.vczt_propagate(_dtype_code(ex), _ptr(ex), _ptr(ey), _ptr(ox), _ptr(oy), _ptr(oz),
                                ctypes.byref(_lib.grid(grid_in)), ctypes.byref(_lib.grid(window)), float(wavelength),
                                float(z), _lens(lens), b, _stream(ex))
    _lib.check("vczt_propagate", st)
    return ox, oy, oz


def vczt_adjoint(gx, gy, gz, grid_in, window, wavelength, z=0.0, lens=None):
    lib = library()
    _field(gx, "gx")
    b = _batch(gx, window)
    _arg(gy, "gy", gx, window, b), _arg(gz, "gz", gx, window, b)
    gex, gey = _like(gx, grid_in, None), _like(gx, grid_in, None)
    with torch.cuda.device(gx.device):
        st = lib.vczt_adjoint(_dtype_code(gx), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gex), _ptr(gey),
                              ctypes.byref(_lib.grid(grid_in)), ctypes.byref(_lib.grid(window)), float(wavelength),
                              float(z), _lens(lens), b, _stream(gx))
    _lib.check("vczt_adjoint", st)
    return gex, gey


# ---------------------------------------------------------- sources, elements --

def prop_source_gaussian(grid, w0, wavelength, amplitude=1.0, lens_f=0.0, batch=1, dtype=torch.complex64,
                         device="cuda"):
    lib = library()
    out = torch.empty((batch, int(grid.ny), int(grid.nx)), dtype=dtype, device=device)
    with torch.cuda.device(out.device):
        st = lib.prop_source_gaussian(_dtype_code(out), _ptr(out), ctypes.byref(_lib.grid(grid)), float(w0),
                                      float(amplitude), float(lens_f), float(wavelength), batch, _stream(out))
    _lib.check("prop_source_gaussian", st)
    return out


def prop_source_radial(grid, w0, batch=1, dtype=torch.complex64, device="cuda"):
    lib = library()
    ex = torch.empty((batch, int(grid.ny), int(grid.nx)), dtype=dtype, device=device)
    ey = torch.empty_like(ex)
    with torch.cuda.device(ex.device):
        st = lib.prop_source_radial(_dtype_code(ex), _ptr(ex), _ptr(ey), ctypes.byref(_lib.grid(grid)), float(w0),
                                    batch, _stream(ex))
    _lib.check("prop_source_radial", st)
    return ex, ey


def prop_modulate(u, phase, out=None):
    """u * exp(i phase); phase [..., ny, nx] (real) broadcast over the batch if it has one item."""
    lib = library()
    _field(u)
    pl = _Plane(u)
    npix = pl.nx * pl.ny
    batch = u.numel() // npix
    _arg(phase, "phase", u, pl, None, real=True)
    pb = phase.numel() // npix
    if pb not in (1, batch):
        raise ValueError(f"phase: {pb} planes, expected 1 or {batch}")
    out = torch.empty_like(u) if out is None else _arg(out, "out", u, pl, batch)
    with torch.cuda.device(u.device):
        st = lib.prop_modulate(_dtype_code(u), _ptr(u), _ptr(phase), _ptr(out), npix, batch, pb, _stream(u))
    _lib.check("prop_modulate", st)
    return out


def prop_modulate_adjoint(g, phase, out=None):
    """g * exp(-i phase): the adjoint of prop_modulate (same broadcasting)."""
    lib = library()
    _field(g, "g")
    pl = _Plane(g)
    npix = pl.nx * pl.ny
    batch = g.numel() // npix
    _arg(phase, "phase", g, pl, None, real=True)
    pb = phase.numel() // npix
    if pb not in (1, batch):
        raise ValueError(f"phase: {pb} planes, expected 1 or {batch}")
    out = torch.empty_like(g) if out is None else _arg(out, "out", g, pl, batch)
    with torch.cuda.device(g.device):
        st = lib.prop_modulate_adjoint(_dtype_code(g), _ptr(g), _ptr(phase), _ptr(out), npix, batch, pb, _stream(g))
    _lib.check("prop_modulate_adjoint", st)
    return out


def prop_phase_grad_sum(g_u, u, grad=None, accumulate=False):
    """sum over the batch of Im(g_u conj(u)): the gradient of a phase shared
    by all batch items (real [ny, nx])."""
    lib = library()
    _field(u)
    pl = _Plane(u)
    npix = pl.nx * pl.ny
    batch = u.numel() // npix
    _arg(g_u, "g_u", u, pl, batch)
    if grad is None:
        grad = torch.empty(tuple(u.shape[-2:]), dtype=_real_dtype(u), device=u.device)
    _arg(grad, "grad", u, pl, 1, real=True)
    with torch.cuda.device(u.device):
        st = lib.prop_phase_grad_sum(_dtype_code(u), _ptr(g_u), _ptr(u), _ptr(grad), npix,
                                     batch, 1 if accumulate else 0, _stream(u))
    _lib.check("prop_phase_grad_sum", st)
    return grad


def prop_scale_items(planes, scale, out=None):
    """Each plane's batch item b times scale[b] (float64 [batch]); into new
    planes, or into `out` (which may be `planes`: in place)."""
    lib = library()
    planes = [t.contiguous() for t in planes]
    ref = _field(planes[0], "planes[0]")
    pl = _Plane(ref)
    npix = pl.nx * pl.ny
    batch = ref.numel() // npix
    for k, t in enumerate(planes):
        _arg(t, f"planes[{k}]", ref, pl, batch)
    scale = scale.to(torch.float64).contiguous()
    _arg(scale, "scale", ref, dtype=torch.float64)
    if scale.numel() != batch:
        raise ValueError("scale must have one entry per batch item")
    out = [torch.empty_like(t) for t in planes] if out is None else list(out)
    if len(out) != len(planes):
        raise ValueError("out must hold one plane per input plane")
    for k, t in enumerate(out):
        _arg(t, f"out[{k}]", ref, pl, batch)
    with torch.cuda.device(ref.device):
        st = lib.prop_scale_items(_dtype_code(ref), _ptr_array(planes), _ptr_array(out), len(planes), _ptr(scale),
                                  npix, batch, _stream(ref))
    _lib.check("prop_scale_items", st)
    return out


def prop_phase_grad(g_u, u, grad=None, accumulate=False):
    """Im(g_u conj(u)) (real, same shape as u)."""
    lib = library()
    _field(u)
    pl = _Plane(u)
    npix = pl.nx * pl.ny
    batch = u.numel() // npix
    _arg(g_u, "g_u", u, pl, batch)
    if grad is None:
        grad = torch.empty(u.shape, dtype=_real_dtype(u), device=u.device)
    _arg(grad, "grad", u, pl, batch, real=True)
    with torch.cuda.device(u.device):
        st = lib.prop_phase_grad(_dtype_code(u), _ptr(g_u), _ptr(u), _ptr(grad), npix, batch, int(accumulate),
                                 _stream(u))
    _lib.check("prop_phase_grad", st)
    return grad


def prop_waveplate(ex, ey, eta, theta):
    lib = library()
    _field(ex, "ex")
    pl = _Plane(ex)
    npix = pl.nx * pl.ny
    batch = ex.numel() // npix
    _arg(ey, "ey", ex, pl, batch)
    ox, oy = torch.empty_like(ex), torch.empty_like(ey)
    with torch.cuda.device(ex.device):
        st = lib.prop_waveplate(_dtype_code(ex), _ptr(ex), _ptr(ey), _ptr(ox), _ptr(oy), float(eta), float(theta),
                                npix, batch, _stream(ex))
    _lib.check("prop_waveplate", st)
    return ox, oy


def prop_waveplate_adjoint(gx, gy, ex, ey, eta, theta):
    """Returns (g_ex, g_ey, dparams[batch, 2] = (dL/deta, dL/dtheta))."""
    lib = library()
    _field(ex, "ex")
    pl = _Plane(ex)
    npix = pl.nx * pl.ny
    batch = ex.numel() // npix
    _arg(ey, "ey", ex, pl, batch), _arg(gx, "gx", ex, pl, batch), _arg(gy, "gy", ex, pl, batch)
    gex, gey = torch.empty_like(gx), torch.empty_like(gy)
    dp = torch.empty((batch, 2), dtype=torch.float64, device=ex.device)
    with torch.cuda.device(ex.device):
        st = lib.prop_waveplate_adjoint(_dtype_code(ex), _ptr(gx), _ptr(gy), _ptr(ex), _ptr(ey), _ptr(gex),
                                        _ptr(gey), float(eta), float(theta), _ptr(dp), npix, batch, _stream(ex))
    _lib.check("prop_waveplate_adjoint", st)
    return gex, gey, dp


def _items(t, npix):
    return t.numel() // npix


def prop_waveplate_batched(ex, ey, params, out=None):
    """Wave plates with one (eta, theta) per batch item: params float64
    [batch, 2] on the fields' device.  Returns (ox, oy), written into
    out = (ox, oy) when given."""
    lib = library()
    ex, ey, params = ex.contiguous(), ey.contiguous(), params.contiguous()
    _field(ex, "ex")
    pl = _Plane(ex)
    npix = pl.nx * pl.ny
    batch = _items(ex, npix)
    _arg(ey, "ey", ex, pl, batch)
    _arg(params, "params", ex, dtype=torch.float64)
    if params.numel() != 2 * batch:
        raise ValueError("params must be float64 [batch, 2]")
    if out is None:
        ox, oy = torch.empty_like(ex), torch.empty_like(ey)
    else:
        ox, oy = _arg(out[0], "out[0]", ex, pl, batch), _arg(out[1], "out[1]", ex, pl, batch)
    with torch.cuda.device(ex.device):
        st = lib.prop_waveplate_batched(_dtype_code(ex), _ptr(ex), _ptr(ey), _ptr(ox), _ptr(oy), _ptr(params), npix,
                                        batch, _stream(ex))
    _lib.check("prop_waveplate_batched", st)
    return ox, oy


def prop_waveplate_batched_adjoint(gx, gy, ex, ey, params, grad=True, shared_input=False, out=None):
    """Returns (g_ex, g_ey, dparams[batch, 2] float64 or None).  With
    shared_input (the plate was fed one field on both components) it returns
    (g_A, None, dparams), g_A = g_ex + g_ey.  out = (g_ex, g_ey) (g_ey None
    with shared_input) receives the field gradients when given."""
    lib = library()
    gx, gy, params = gx.contiguous(), gy.contiguous(), params.contiguous()
    _field(gx, "gx")
    pl = _Plane(gx)
    npix = pl.nx * pl.ny
    batch = _items(gx, npix)
    _arg(gy, "gy", gx, pl, batch)
    _arg(params, "params", gx, dtype=torch.float64)
    if params.numel() != 2 * batch:
        raise ValueError("params must be float64 [batch, 2]")
    if out is None:
        gex = torch.empty_like(gx)
        gey = None if shared_input else torch.empty_like(gy)
    else:
        gex = _arg(out[0], "out[0]", gx, pl, batch)
        gey = None if shared_input else _arg(out[1], "out[1]", gx, pl, batch)
    dp = torch.empty((batch, 2), dtype=torch.float64, device=gx.device) if grad else None
    if grad:
        ex, ey = ex.contiguous(), ey.contiguous()
        _arg(ex, "ex", gx, pl, batch), _arg(ey, "ey", gx, pl, batch)
    with torch.cuda.device(gx.device):
        st = lib.prop_waveplate_batched_adjoint(_dtype_code(gx), _ptr(gx), _ptr(gy), _ptr(ex) if grad else None,
                                                _ptr(ey) if grad else None, _ptr(gex),
                                                _ptr(gey) if gey is not None else None, _ptr(params),
                                                _ptr(dp) if grad else None, npix, batch, _stream(gx))
    _lib.check("prop_waveplate_batched_adjoint", st)
    return gex, gey, dp


def _port(planes):
    return None if planes is None else [t.contiguous() for t in planes]


def prop_beam_splitter(a, b, alpha, out=None):
    """Beam splitter with one mixing angle per batch item (alpha float64
    [batch]): a, b are lists of component planes [batch, ny, nx] (or None:
    dark port).  Returns (c, d) as lists of planes, written into
    out = (c, d) when given."""
    lib = library()
    a, b = _port(a), _port(b)
    if not (a or b):
        raise ValueError("at least one input port must carry a field")
    ref = _field((a or b)[0], "port")
    ncomp = len(a or b)
    if a and b and len(a) != len(b):
        raise ValueError("both ports must have the same number of components")
    pl = _Plane(ref)
    npix = pl.nx * pl.ny
    batch = _items(ref, npix)
    for k, t in enumerate((a or []) + (b or [])):
        _arg(t, f"port plane {k}", ref, pl, batch)
    alpha = alpha.contiguous()
    _arg(alpha, "alpha", ref, dtype=torch.float64)
    if alpha.numel() != batch:
        raise ValueError("alpha must be float64 [batch]")
    if out is None:
        c = [torch.empty_like(ref) for _ in range(ncomp)]
        d = [torch.empty_like(ref) for _ in range(ncomp)]
    else:
        c, d = list(out[0]), list(out[1])
        if len(c) != ncomp or len(d) != ncomp:
            raise ValueError(f"out: {ncomp} planes per output port expected")
        for k, t in enumerate(c + d):
            _arg(t, f"out plane {k}", ref, pl, batch)
    with torch.cuda.device(ref.device):
        st = lib.prop_beam_splitter(_dtype_code(ref), _ptr_array(a) if a else None, _ptr_array(b) if b else None,
                                    _ptr_array(c), _ptr_array(d), ncomp, _ptr(alpha), npix, batch, _stream(ref))
    _lib.check("prop_beam_splitter", st)
    return c, d


def prop_beam_splitter_adjoint(gc, gd, a, b, alpha, want=(True, True), grad=True, out=None):
    """Returns (g_a or None, g_b or None, dalpha[batch] float64 or None);
    a, b are the forward inputs (None: dark), needed only for dalpha.
    out = (g_a, g_b) (plane lists, the entry of an unwanted port ignored)
    receives the port gradients when given."""
    lib = library()
    gc, gd = _port(gc), _port(gd)
    a, b = _port(a), _port(b)
    ref, ncomp = _field(gc[0], "gc[0]"), len(gc)
    pl = _Plane(ref)
    npix = pl.nx * pl.ny
    batch = _items(ref, npix)
    if len(gd) != ncomp or (a and len(a) != ncomp) or (b and len(b) != ncomp):
        raise ValueError("every port must have the same number of components")
    for k, t in enumerate(gc + gd + (a or []) + (b or [])):
        _arg(t, f"port plane {k}", ref, pl, batch)
    alpha = alpha.contiguous()
    _arg(alpha, "alpha", ref, dtype=torch.float64)
    if alpha.numel() != batch:
        raise ValueError("alpha must be float64 [batch]")
    if out is None:
        ga = [torch.empty_like(ref) for _ in range(ncomp)] if want[0] else None
        gb = [torch.empty_like(ref) for _ in range(ncomp)] if want[1] else None
    else:
        ga = list(out[0]) if want[0] else None
        gb = list(out[1]) if want[1] else None
        if (ga and len(ga) != ncomp) or (gb and len(gb) != ncomp):
            raise ValueError(f"out: {ncomp} planes per wanted port expected")
        for k, t in enumerate((ga or []) + (gb or [])):
            _arg(t, f"out plane {k}", ref, pl, batch)
    da = torch.empty((batch,), dtype=torch.float64, device=ref.device) if grad else None
    with torch.cuda.device(ref.device):
        st = lib.prop_beam_splitter_adjoint(_dtype_code(ref), _ptr_array(gc), _ptr_array(gd),
                                            _ptr_array(a) if a else None, _ptr_array(b) if b else None,
                                            _ptr_array(ga) if ga else None, _ptr_array(gb) if gb else None, ncomp,
                                            _ptr(alpha), _ptr(da) if grad else None, npix, batch, _stream(ref))
    _lib.check("prop_beam_splitter_adjoint", st)
    return ga, gb, da


def prop_spot_loss(ex, ey, ez, window, wavelength, w_fz=0.0, seeds=True, noalloc=False):
    """Returns (result[batch, 8] float64, (g_x, g_y, g_z) or None).

    result columns: loss, sigma^2, F_z, P, Xbar - cx, Ybar - cy, 0, 0.
    noalloc=True calls prop_spot_loss_noalloc (no device allocation in the
    library; batch <= 256).
    """
    lib = library()
    _field(ex, "ex")
    b = _batch(ex, window)
    _arg(ey, "ey", ex, window, b)
    if ez is not None:
        _arg(ez, "ez", ex, window, b)
    res = torch.empty((b, 8), dtype=torch.float64, device=ex.device)
    gx = gy = gz = None
    if seeds:
        gx, gy = torch.empty_like(ex), torch.empty_like(ey)
        gz = torch.empty_like(ez) if ez is not None else None
    fn = lib.prop_spot_loss_noalloc if noalloc else lib.prop_spot_loss
    with torch.cuda.device(ex.device):
        st = fn(_dtype_code(ex), _ptr(ex), _ptr(ey), _ptr(ez), ctypes.byref(_lib.grid(window)), float(wavelength),
                float(w_fz), _ptr(res), _ptr(gx), _ptr(gy), _ptr(gz), b, _stream(ex))
    _lib.check("prop_spot_loss_noalloc" if noalloc else "prop_spot_loss", st)
    return res, ((gx, gy, gz) if seeds else None)


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * max(len(tensors), 1))()
    for k, t in enumerate(tensors):
        arr[k] = t.data_ptr() if t is not None else None
    return arr


def prop_density_loss(comps, eps, dep=None, beta=1.0, seeds=True):
    """Threshold-density loss Area / I_eps of the intensity of `comps` (STED-
    modulated by `dep` if given).  Returns (result[batch, 4] float64 =
    (loss, area, I_eps, max I), seeds for comps, seeds for dep)."""
    lib = library()
    comps = [c.contiguous() for c in comps]
    dep = [d.contiguous() for d in (dep or [])]
    ref = _field(comps[0], "comps[0]")
    pl = _Plane(ref)
    npix = pl.nx * pl.ny
    batch = ref.numel() // npix
    for k, t in enumerate(comps + dep):
        _arg(t, f"component {k}", ref, pl, batch)
    res = torch.empty((batch, 4), dtype=torch.float64, device=ref.device)
    gs = [torch.empty_like(c) for c in comps] if seeds else []
    gd = [torch.empty_like(d) for d in dep] if seeds else []
    with torch.cuda.device(ref.device):
        st = lib.prop_density_loss(_dtype_code(ref), _ptr_array(comps), len(comps), _ptr_array(dep), len(dep),
                                   float(beta), npix, float(eps), _ptr(res), _ptr_array(gs) if seeds else None,
                                   _ptr_array(gd) if (seeds and dep) else None, batch, _stream(ref))
    _lib.check("prop_density_loss", st)
    return res, gs, gd


def prop_softmin(losses, beta):
    """Smooth minimum over the last axis of float64 `losses` [batch, ndet]:
    returns (value[batch], weights[batch, ndet] = d value / d losses)."""
    lib = library()
    losses = losses.contiguous()
    _dev(losses)
    ndet = losses.shape[-1]
    batch = losses.numel() // ndet
    val = torch.empty((batch,), dtype=torch.float64, device=losses.device)
    w = torch.empty((batch, ndet), dtype=torch.float64, device=losses.device)
    with torch.cuda.device(losses.device):
        st = lib.prop_softmin(_ptr(losses), ndet, float(beta), _ptr(val), _ptr(w), batch, _stream(losses))
    _lib.check("prop_softmin", st)
    return val, w


def prop_adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """In-place Adam (AdamW if weight_decay > 0) step on a real float32 or
    float64 device tensor with its gradient and moment buffers."""
    lib = library()
    for t in (param, grad, m, v):
        _dev(t)
        if not t.is_contiguous() or t.dtype != param.dtype or t.numel() != param.numel():
            raise ValueError("param, grad, m, v: contiguous, same dtype and size")
    code = _lib.PROP_C64 if param.dtype == torch.float32 else _lib.PROP_C128
    with torch.cuda.device(param.device):
        st = lib.prop_adam_step(code, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), float(lr),
                                float(beta1), float(beta2), float(eps), float(weight_decay), int(step),
                                _stream(param))
    _lib.check("prop_adam_step", st)


class Adam:
    """Minimal device optimiser over a list of real tensors (phases, retarder
    parameters, distances), stepping with prop_adam_step."""

    def __init__(self, params, lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.0):
        self.params = list(params)
        self.lr, self.betas, self.eps, self.wd = lr, betas, eps, weight_decay
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def step(self):
        self.t += 1
        for p, m, v in zip(self.params, self.m, self.v):
            if p.grad is None:
                continue
            prop_adam_step(p.data, p.grad.contiguous(), m, v, self.t, self.lr, self.betas[0], self.betas[1], self.eps,
                           self.wd)

    def zero_grad(self):
        for p in self.params:
            p.grad = None


def prop_sum_items(x):
    """Sum over the leading (batch) axis of a float64 device tensor, in item
    order on the device: [n, ...] -> [...] (a batch-shared parameter's
    gradient from per-item gradients)."""
    lib = library()
    _dev(x, "x")
    if x.dtype != torch.float64 or x.dim() < 1 or x.shape[0] < 1 or x.numel() < 1:
        raise ValueError("x must be a non-empty float64 [n, ...] tensor")
    n = int(x.shape[0])
    m = x.numel() // n
    out = torch.empty(tuple(x.shape[1:]), dtype=torch.float64, device=x.device)
    with torch.cuda.device(x.device):
        st = lib.prop_sum_items(_ptr(x), _ptr(out), n, m, _stream(x))
    _lib.check("prop_sum_items", st)
    return out


def prop_track_best(loss, best, since):
    """One step of the stopping rule's bookkeeping on the device: per batch
    item, best = loss and since = 0 where loss < best, else since += 1.
    loss, best: float64 [B]; since: int64 [B] (updated in place)."""
    lib = library()
    for t, dt in ((loss, torch.float64), (best, torch.float64), (since, torch.int64)):
        _dev(t)
        if t.dtype != dt or not t.is_contiguous() or t.numel() != loss.numel():
            raise ValueError("loss, best: float64 [B]; since: int64 [B]; contiguous")
    with torch.cuda.device(loss.device):
        st = lib.prop_track_best(_ptr(loss), _ptr(best), _ptr(since), loss.numel(), _stream(loss))
    _lib.check("prop_track_best", st)


class StopRule:
    """The paper's stopping condition: every `check_every` steps, stop if
    the best objective so far is `patience` or more steps old (500 and 100
    in its discovery runs).  The best value and the steps
    since it fell stay on the device; `update` reads them back only at
    checks.  With a batch of objectives, `update` reports True once every
    item has stalled; `stalled` gives the per-item state of the last check."""

    def __init__(self, patience=500, check_every=100, batch=1, device="cuda"):
        if patience < 1 or check_every < 1:
            raise ValueError("patience and check_every must be positive")
        self.patience, self.check_every = int(patience), int(check_every)
        self.best = torch.full((batch,), float("inf"), dtype=torch.float64, device=device)
        self.since = torch.zeros(batch, dtype=torch.int64, device=device)
        self.steps = 0
        self.stalled = torch.zeros(batch, dtype=torch.bool)

    def update(self, loss) -> bool:
        loss = loss.detach().reshape(-1)
        if loss.dtype != torch.float64:
            loss = loss.to(torch.float64)
        prop_track_best(loss.contiguous(), self.best, self.since)
        self.steps += 1
        if self.steps % self.check_every:
            return False
        self.stalled = self.since.cpu() >= self.patience
        return bool(self.stalled.all())


def prop_sampling_check(grid, wavelength, z) -> int:
    return library().prop_sampling_check(ctypes.byref(_lib.grid(grid)), float(wavelength), float(z))


def prop_fft_length(n: int) -> int:
    return library().prop_fft_length(int(n))


def prop_cache_clear() -> None:
    library().prop_cache_clear()


def prop_cache_set_limit(nbytes: int) -> None:
    """Byte budget of the cached kernel spectra and zoom vectors (<= 0: default)."""
    library().prop_cache_set_limit(int(nbytes))


def prop_cache_info() -> dict:
    """Snapshot of the table cache (bytes, limit, entries, pins, evictions)."""
    st = _lib.prop_cache_stats()
    library().prop_cache_info(ctypes.byref(st))
    return {name: int(getattr(st, name)) for name, _ in _lib.prop_cache_stats._fields_}


def prop_trace_enable(on: bool = True) -> None:
    library().prop_trace_enable(1 if on else 0)


def prop_trace_only(name=None) -> None:
    """Trace only the launches of pass `name` (None: every pass again)."""
    library().prop_trace_only(None if name is None else str(name).encode())


def prop_trace_read(max_entries: int = 64) -> dict:
    """{pass name: (launches, total_ms, bytes)} of the trace since enable (clears it)."""
    lib = library()
    buf = (_lib.prop_trace_stat * max_entries)()
    n = lib.prop_trace_read(ctypes.cast(buf, ctypes.c_void_p), max_entries)
    if n < 0:
        raise PropError("prop_trace_read", n)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms), float(buf[i].bytes))
            for i in range(n)}


def prop_tune_cache_path(path=None) -> int:
    """Set the tuning cache file (None: the default) and read it; returns the
    number of usable records."""
    return int(library().prop_tune_cache_path(None if path is None else os.fsencode(path)))


def prop_tune_cache_rejected() -> int:
    """Lines of the tuning cache file skipped as malformed or unusable."""
    return int(library().prop_tune_cache_rejected())


def prop_autotune_report() -> str:
    """One line per shape the autotuner has tuned (chosen variant, ms of each)."""
    lib = library()
    need = lib.prop_autotune_report(None, 0)
    buf = ctypes.create_string_buffer(max(int(need), 1))
    lib.prop_autotune_report(buf, len(buf))
    return buf.value.decode()


# ---------------------------------------------------------------------- plans --

PROP_OP_RS, PROP_OP_CZT, PROP_OP_VRS, PROP_OP_VCZT, PROP_OP_RS_CZT = 0, 1, 2, 3, 4
PROP_PLAN_GRAPH = 1
PROP_PLAN_AUTOTUNE = 2
PROP_PLAN_FAULT_NOMEM = 0x100


class Setup:
    """One propagator call of a plan (see prop_setup in include/libprop.h).

    Tensors are device tensors of the plan's dtype; ``inputs``/``outputs``/
    ``grad_outputs``/``grad_inputs`` are lists (1 or 2 inputs, 1 or 3 outputs).
    """

    def __init__(self, op, grid, inputs, outputs, grad_outputs, wavelength, z=0.0, window=None, lens=None,
                 lens_f=0.0, phase=None, grad_inputs=None, grad_phase=None, z2=0.0):
        self.op, self.grid, self.window = op, grid, window
        self.z2 = z2
        self.inputs, self.outputs, self.grad_outputs = list(inputs), list(outputs), list(grad_outputs)
        self.grad_inputs = list(grad_inputs) if grad_inputs is not None else []
        self.wavelength, self.z, self.lens, self.lens_f = wavelength, z, lens, lens_f
        self.phase, self.grad_phase = phase, grad_phase

    def _struct(self, dtype, device):
        """The prop_setup of this setup, after checking every tensor against
        the plan's dtype and device and the setup's grids and batch."""
        vec = self.op in (PROP_OP_VRS, PROP_OP_VCZT)
        nin, nout = (2, 3) if vec else (1, 1)
        if self.op not in (PROP_OP_RS, PROP_OP_CZT, PROP_OP_VRS, PROP_OP_VCZT, PROP_OP_RS_CZT):
            raise ValueError(f"unknown op {self.op}")
        if len(self.inputs) != nin or len(self.outputs) != nout or len(self.grad_outputs) != nout:
            raise ValueError(f"op {self.op} takes {nin} inputs, {nout} outputs and {nout} output gradients")
        if self.grad_inputs and len(self.grad_inputs) != nin:
            raise ValueError(f"op {self.op} takes {nin} input gradients")
        ref = _field(self.inputs[0], "inputs[0]")
        if ref.dtype != dtype:
            raise ValueError(f"setup dtype {ref.dtype} differs from the plan's {dtype}")
        if ref.device != device:
            raise ValueError(f"setup tensors on {ref.device}, the plan runs on {device}")
        b = _batch(ref, self.grid)
        out_grid = self.window if self.op in (PROP_OP_CZT, PROP_OP_VCZT, PROP_OP_RS_CZT) else self.grid
        if out_grid is None:
            raise ValueError("CZT, VCZT and RS_CZT setups need an output window")
        for name, ts, g in (("inputs", self.inputs, self.grid), ("outputs", self.outputs, out_grid),
                            ("grad_outputs", self.grad_outputs, out_grid), ("grad_inputs", self.grad_inputs, self.grid)):
            for i, t in enumerate(ts):
                if t is not None:
                    _arg(t, f"{name}[{i}]", ref, g, b)
        for name, t in (("phase", self.phase), ("grad_phase", self.grad_phase)):
            if t is not None:
                _arg(t, name, ref, self.grid, b, real=True)
        s = _lib.prop_setup()
        s.op = self.op
        s.batch = b
        s.g_in = _lib.grid(self.grid)
        if self.window is not None:
            s.win = _lib.grid(self.window)
        s.wavelength, s.z, s.z2 = float(self.wavelength), float(self.z), float(self.z2)
        if self.lens is not None:
            na, f = (self.lens.na, self.lens.f) if hasattr(self.lens, "na") else self.lens
            s.has_lens, s.lens = 1, _lib.prop_lens(float(na), float(f))
        s.lens_f = float(self.lens_f)
        s.phase = self.phase.data_ptr() if self.phase is not None else None
        for i, t in enumerate(self.inputs):
            s.in_[i] = t.data_ptr()
        for i, t in enumerate(self.outputs):
            s.out[i] = t.data_ptr()
        for i, t in enumerate(self.grad_outputs):
            s.gout[i] = t.data_ptr()
        for i, t in enumerate(self.grad_inputs):
            s.gin[i] = t.data_ptr() if t is not None else None
        s.grad_phase = self.grad_phase.data_ptr() if self.grad_phase is not None else None
        return s


class Plan:
    """A prop_plan over a list of Setups (keeps their tensors alive)."""

    def __init__(self, setups, dtype=torch.complex64, graph=False, device=None, autotune=False, flags=0):
        lib = library()
        self.setups = list(setups)
        if not self.setups:
            raise ValueError("a plan needs at least one setup")
        if dtype not in (torch.complex64, torch.complex128):
            raise TypeError(f"plan dtype must be complex64 or complex128, got {dtype}")
        self.device = torch.device(device) if device is not None else self.setups[0].inputs[0].device
        arr = (_lib.prop_setup * len(self.setups))(*[s._struct(dtype, self.device) for s in self.setups])
        self._arr = arr
        h = ctypes.c_void_p()
        code = _lib.PROP_C64 if dtype == torch.complex64 else _lib.PROP_C128
        fl = (PROP_PLAN_GRAPH if graph else 0) | (PROP_PLAN_AUTOTUNE if autotune else 0) | int(flags)
        with torch.cuda.device(self.device):
            st = lib.prop_plan_create(code, ctypes.cast(arr, ctypes.c_void_p), len(self.setups), fl,
                                      ctypes.byref(h))
        _lib.check("prop_plan_create", st)
        self._h = h

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self):
        with torch.cuda.device(self.device):
            _lib.check("prop_plan_forward", library().prop_plan_forward(self._h, self._stream()))

    def adjoint(self):
        with torch.cuda.device(self.device):
            _lib.check("prop_plan_adjoint", library().prop_plan_adjoint(self._h, self._stream()))

    def step(self):
        """forward() then adjoint(), as one graph launch for a graph plan."""
        with torch.cuda.device(self.device):
            _lib.check("prop_plan_step", library().prop_plan_step(self._h, self._stream()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().prop_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
