"""ctypes binding of libprop.so: signatures and status handling only.

``torch`` is imported before the library is loaded so that the library
binds to the HIP runtime torch already loaded (same soname), which makes
torch's device pointers and streams valid inside the library.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import torch  # noqa: F401  (must precede loading libprop.so)

HERE = os.path.dirname(os.path.abspath(__file__))
# LIBPROP_PATH selects another build of the same library (the host-sanitized
# variant of the ABI tests); by default the in-tree libprop.so.
LIB_PATH = os.environ.get("LIBPROP_PATH") or os.path.join(HERE, "libprop.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = c_void_p

PROP_C64, PROP_C128 = 0, 1
STATUS = {0: "PROP_OK", 1: "PROP_WUNDERSAMPLED", -1: "PROP_ENULL", -2: "PROP_ESHAPE", -3: "PROP_EPARAM",
          -4: "PROP_EALIAS", -5: "PROP_ENOMEM", -6: "PROP_EDEVICE", -7: "PROP_ELIMIT"}


class prop_grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("dx", c_double), ("dy", c_double),
                ("cx", c_double), ("cy", c_double)]


class prop_lens(ctypes.Structure):
    _fields_ = [("na", c_double), ("f", c_double)]


class prop_trace_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int32), ("total_ms", c_double), ("bytes", c_double)]


class prop_setup(ctypes.Structure):
    _fields_ = [("op", c_int32), ("batch", c_int32), ("g_in", prop_grid), ("win", prop_grid),
                ("wavelength", c_double), ("z", c_double), ("has_lens", c_int32), ("lens", prop_lens),
                ("lens_f", c_double), ("phase", c_void_p), ("in_", c_void_p * 2), ("out", c_void_p * 3),
                ("gout", c_void_p * 3), ("gin", c_void_p * 2), ("grad_phase", c_void_p), ("z2", c_double)]


class prop_cache_stats(ctypes.Structure):
    _fields_ = [("table_bytes", c_int64), ("limit", c_int64), ("spectra", c_int64), ("zooms", c_int64),
                ("twiddles", c_int64), ("pinned", c_int64), ("evictions", c_int64), ("eviction_syncs", c_int64)]


G = ctypes.POINTER(prop_grid)
LENS = ctypes.POINTER(prop_lens)
DPTR = ctypes.POINTER(c_double)

# name -> (restype, argtypes); mirrors include/libprop.h
SIGNATURES = {
    "rs_propagate": (c_int32, [c_int32, P, P, G, c_double, c_double, c_int32, P]),
    "rs_adjoint": (c_int32, [c_int32, P, P, G, c_double, c_double, c_int32, P]),
    "czt_propagate": (c_int32, [c_int32, P, P, G, G, c_double, c_double, c_int32, P]),
    "czt_adjoint": (c_int32, [c_int32, P, P, G, G, c_double, c_double, c_int32, P]),
    "vrs_propagate": (c_int32, [c_int32, P, P, P, P, P, G, c_double, c_double, c_int32, P]),
    "vrs_adjoint": (c_int32, [c_int32, P, P, P, P, P, G, c_double, c_double, c_int32, P]),
    "vczt_propagate": (c_int32, [c_int32, P, P, P, P, P, G, G, c_double, c_double, LENS, c_int32, P]),
    "vczt_adjoint": (c_int32, [c_int32, P, P, P, P, P, G, G, c_double, c_double, LENS, c_int32, P]),
    "prop_source_gaussian": (c_int32, [c_int32, P, G, c_double, c_double, c_double, c_double, c_int32, P]),
    "prop_source_radial": (c_int32, [c_int32, P, P, G, c_double, c_int32, P]),
    "prop_modulate": (c_int32, [c_int32, P, P, P, c_int64, c_int32, c_int32, P]),
    "prop_modulate_adjoint": (c_int32, [c_int32, P, P, P, c_int64, c_int32, c_int32, P]),
    "prop_phase_grad_sum": (c_int32, [c_int32, P, P, P, c_int64, c_int32, c_int32, P]),
    "prop_scale_items": (c_int32, [c_int32, P, P, c_int32, P, c_int64, c_int32, P]),
    "prop_phase_grad": (c_int32, [c_int32, P, P, P, c_int64, c_int32, c_int32, P]),
    "prop_waveplate": (c_int32, [c_int32, P, P, P, P, c_double, c_double, c_int64, c_int32, P]),
    "prop_waveplate_adjoint": (c_int32, [c_int32, P, P, P, P, P, P, c_double, c_double, P, c_int64, c_int32, P]),
    "prop_waveplate_batched": (c_int32, [c_int32, P, P, P, P, P, c_int64, c_int32, P]),
    "prop_waveplate_batched_adjoint": (c_int32, [c_int32, P, P, P, P, P, P, P, P, c_int64, c_int32, P]),
    "prop_beam_splitter": (c_int32, [c_int32, P, P, P, P, c_int32, P, c_int64, c_int32, P]),
    "prop_beam_splitter_adjoint": (c_int32, [c_int32, P, P, P, P, P, P, c_int32, P, P, c_int64, c_int32, P]),
    "prop_spot_loss": (c_int32, [c_int32, P, P, P, G, c_double, c_double, P, P, P, P, c_int32, P]),
    "prop_spot_loss_noalloc": (c_int32, [c_int32, P, P, P, G, c_double, c_double, P, P, P, P, c_int32, P]),
    "prop_sampling_check": (c_int32, [G, c_double, c_double]),
    "prop_fft_length": (c_int32, [c_int32]),
    "prop_cache_clear": (None, []),
    "prop_cache_set_limit": (None, [c_int64]),
    "prop_cache_info": (None, [P]),
    "prop_status_string": (ctypes.c_char_p, [c_int32]),
    "prop_last_device_error": (c_int32, []),
    "prop_plan_create": (c_int32, [c_int32, P, c_int32, ctypes.c_uint32, ctypes.POINTER(c_void_p)]),
    "prop_plan_forward": (c_int32, [P, P]),
    "prop_plan_adjoint": (c_int32, [P, P]),
    "prop_plan_step": (c_int32, [P, P]),
    "prop_plan_destroy": (None, [P]),
    "prop_trace_enable": (None, [c_int32]),
    "prop_trace_read": (c_int32, [P, c_int32]),
    "prop_trace_only": (None, [ctypes.c_char_p]),
    "prop_autotune_report": (c_int32, [ctypes.c_char_p, c_int32]),
    "prop_tune_cache_path": (c_int32, [ctypes.c_char_p]),
    "prop_tune_cache_rejected": (c_int32, []),
    "rs_grad_z": (c_int32, [c_int32, P, P, P, G, c_double, c_double, c_int32, P]),
    "rs_adjoint_grad_z": (c_int32, [c_int32, P, P, P, P, G, c_double, c_double, c_int32, P]),
    "rs_adjoint_phase_grad": (c_int32, [c_int32, P, P, P, P, c_int32, G, c_double, c_double, c_int32, P]),
    "czt_adjoint_phase_grad": (c_int32, [c_int32, P, P, P, P, c_int32, G, G, c_double, c_double, c_int32, P]),
    "czt_grad_z": (c_int32, [c_int32, P, P, P, P, G, G, c_double, c_double, c_int32, P]),
    "prop_density_loss": (c_int32, [c_int32, P, c_int32, P, c_int32, c_double, c_int64, c_double, P, P, P, c_int32,
                                     P]),
    "prop_softmin": (c_int32, [P, c_int32, c_double, P, P, c_int32, P]),
    "prop_track_best": (c_int32, [P, P, P, c_int32, P]),
    "prop_sum_items": (c_int32, [P, P, c_int32, c_int32, P]),
    "prop_adam_step": (c_int32, [c_int32, P, P, P, P, c_int64, c_double, c_double, c_double, c_double, c_double,
                                 c_int32, P]),
}

_lib = None


class PropError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        msg = _lib.prop_status_string(status).decode() if _lib is not None else STATUS.get(status, "?")
        extra = ""
        if status == -6 and _lib is not None:
            extra = f" (hipError {_lib.prop_last_device_error()})"
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}{extra}")


class PropWarning(UserWarning):
    pass


def load():
    """Load libprop.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libprop.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                           "or python -m paper_2310_08408_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(fn: str, status: int) -> int:
    if status < 0:
        raise PropError(fn, status)
    if status > 0:
        warnings.warn(f"{fn}: {STATUS.get(status, status)}", PropWarning, stacklevel=3)
    return status


def grid(g) -> prop_grid:
    """prop_grid from any object with nx, ny, dx, dy, cx, cy (cx, cy default 0)."""
    return prop_grid(int(g.nx), int(g.ny), float(g.dx), float(g.dy),
                     float(getattr(g, "cx", 0.0)), float(getattr(g, "cy", 0.0)))
