"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/libprop.h declares, the Python signature table mirrors the header,
and argument validation rejects bad calls before any device work.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libprop.h")
LIB = os.environ.get("LIBPROP_PATH") or os.path.join(ROOT, "paper_2310_08408_amd", "libprop.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libprop.so not built")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^(?:int|void|int32_t|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2310_08408_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_signature_table_matches_header():
    from paper_2310_08408_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared()


def _grid(nx=64, ny=64, d=1e-6):
    from paper_2310_08408_amd import _lib
    return _lib.prop_grid(nx, ny, d, d, 0.0, 0.0)


def test_validation_without_device(lib):
    from paper_2310_08408_amd import _lib
    g = _grid()
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x100000000)
    ref = ctypes.byref
    # null pointers
    assert lib.rs_propagate(0, None, out, ref(g), 500e-9, 1e-3, 1, None) == -1
    # bad dtype, wavelength, distance
    assert lib.rs_propagate(7, fake, out, ref(g), 500e-9, 1e-3, 1, None) == -3
    assert lib.rs_propagate(0, fake, out, ref(g), -1.0, 1e-3, 1, None) == -3
    assert lib.rs_propagate(0, fake, out, ref(g), 500e-9, 0.0, 1, None) == -3
    assert lib.rs_propagate(0, fake, out, ref(g), 500e-9, float("nan"), 1, None) == -3
    # bad shapes
    assert lib.rs_propagate(0, fake, out, ref(_grid(0, 4)), 500e-9, 1e-3, 1, None) == -2
    assert lib.rs_propagate(0, fake, out, ref(_grid(5000, 4)), 500e-9, 1e-3, 1, None) == -2
    assert lib.rs_propagate(0, fake, out, ref(g), 500e-9, 1e-3, -1, None) == -2
    # aliasing (in place is rejected)
    assert lib.rs_propagate(0, fake, fake, ref(g), 500e-9, 1e-3, 1, None) == -4
    # empty batch is a no-op (no device work)
    assert lib.rs_propagate(0, None, None, ref(g), 500e-9, 1e-3, 0, None) in (0, 1)
    # CZT: window too large for one transform
    assert lib.czt_propagate(0, fake, out, ref(_grid(6000, 8)), ref(_grid(3000, 8)), 5e-7, 1e-3, 1, None) == -2
    # lens checks
    bad_lens = _lib.prop_lens(1.2, 1e-3)
    assert lib.vczt_propagate(0, fake, fake, out, out, out, ref(g), ref(g), 5e-7, 0.0, ref(bad_lens), 1, None) == -3
    # outputs overlapping each other
    assert lib.vrs_propagate(0, fake, ctypes.c_void_p(0x2000000), out, out, ctypes.c_void_p(0x300000000),
                             ref(g), 5e-7, 1e-2, 1, None) == -4
    assert lib.prop_modulate(0, fake, fake, out, 10, 2, 3, None) == -2
    # distance gradients: z = 0 and a missing output
    assert lib.rs_grad_z(0, fake, fake, out, ref(g), 5e-7, 0.0, 1, None) == -3
    assert lib.czt_grad_z(0, fake, None, fake, None, ref(g), ref(g), 5e-7, 1e-3, 1, None) == -1
    # detector side: component counts, threshold and efficiency ranges, softmin beta
    comps = (ctypes.c_void_p * 3)(fake.value, fake.value, fake.value)
    assert lib.prop_density_loss(0, comps, 0, None, 0, 1.0, 16, 0.5, out, None, None, 1, None) == -2
    assert lib.prop_density_loss(0, comps, 2, None, 4, 1.0, 16, 0.5, out, None, None, 1, None) == -2
    assert lib.prop_density_loss(0, comps, 2, None, 0, 1.0, 16, 1.5, out, None, None, 1, None) == -3
    assert lib.prop_density_loss(0, comps, 2, None, 1, 1.2, 16, 0.5, out, None, None, 1, None) == -3
    assert lib.prop_density_loss(0, comps, 2, None, 1, 1.0, 16, 0.5, out, None, None, 1, None) == -1
    assert lib.prop_softmin(out, 3, 0.0, out, None, 1, None) == -3
    assert lib.prop_softmin(out, 0, 1.0, out, None, 1, None) == -2
    # stopping-rule bookkeeping: batch, missing arrays, best or since on the loss or on each other
    lo, be, si = ctypes.c_void_p(0x70000000), ctypes.c_void_p(0x71000000), ctypes.c_void_p(0x72000000)
    assert lib.prop_track_best(lo, be, si, -1, None) == -2
    assert lib.prop_track_best(lo, be, si, 0, None) == 0     # nothing to do
    assert lib.prop_track_best(lo, None, si, 4, None) == -1
    assert lib.prop_track_best(lo, lo, si, 4, None) == -4
    assert lib.prop_track_best(lo, be, be, 4, None) == -4
    # beam splitter: component count, missing output plane, output on an input
    pa = (ctypes.c_void_p * 2)(0x10000000, 0x20000000)
    pc = (ctypes.c_void_p * 2)(0x30000000, 0x40000000)
    pd = (ctypes.c_void_p * 2)(0x50000000, None)
    pe = (ctypes.c_void_p * 2)(0x60000000, 0x10000000)
    assert lib.prop_beam_splitter(0, pa, None, pc, pc, 0, out, 16, 1, None) == -2
    assert lib.prop_beam_splitter(0, pa, None, pc, pc, 4, out, 16, 1, None) == -2
    assert lib.prop_beam_splitter(0, pa, None, pc, pd, 2, out, 16, 1, None) == -1
    assert lib.prop_beam_splitter(0, pa, None, pc, pe, 2, out, 16, 1, None) == -4
    assert lib.prop_beam_splitter(0, pa, None, None, pc, 2, out, 16, 1, None) == -1
    assert lib.prop_beam_splitter(0, pa, None, pc, pc, 2, out, 0, 1, None) == 0    # nothing to do
    assert lib.prop_beam_splitter_adjoint(0, pa, None, None, None, None, None, 2, out, None, 16, 1, None) == -1
    # per-item wave plates: missing parameters, forward inputs needed for the gradient
    assert lib.prop_waveplate_batched(0, fake, fake, out, out, None, 16, 1, None) == -1
    assert lib.prop_waveplate_batched_adjoint(0, fake, fake, None, None, out, None, fake, out, 16, 1, None) == -1
    assert lib.prop_modulate_adjoint(0, fake, fake, out, 10, 2, 3, None) == -2


def test_lengths_and_sampling(lib):
    assert lib.prop_fft_length(1) == 1
    assert lib.prop_fft_length(255) == 256
    assert lib.prop_fft_length(4095) == 4096
    assert lib.prop_fft_length(2559) == 3072
    assert lib.prop_fft_length(1791) == 2048
    assert lib.prop_fft_length(8193) == -1
    g = _grid(2048, 2048, 4e-3 / 2048)
    assert lib.prop_sampling_check(ctypes.byref(g), 650e-9, 25e-3) == 0
    assert lib.prop_sampling_check(ctypes.byref(g), 650e-9, 20e-3) == 1
    g1 = _grid(128, 128, 1e-3 / 128)
    assert lib.prop_sampling_check(ctypes.byref(g1), 650e-9, 5e-3) == 1


def test_status_strings(lib):
    from paper_2310_08408_amd import _lib
    for code in _lib.STATUS:
        assert lib.prop_status_string(code)
