"""GPU parity of scalar RS and CZT (forward and adjoint) against the FP64
oracle, through the C ABI (via the thin Python binding).

Tolerances: relative L2 <= 1e-5 for FP32 (complex64) fields, <= 1e-12 for
the FP64 (complex128) path.  Inputs are cast to the kernel precision first;
the oracle consumes the cast values upcast to complex128.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import Grid
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    return lp


def dev(a, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def cast(a, kind):
    return np.asarray(a, np.complex64 if kind == "c64" else np.complex128).astype(np.complex128)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rnd(shape, seed):
    rng = np.random.default_rng(seed)
    return workloads.random_field(rng, shape)


# ------------------------------------------------------------------- RS --

def test_rs_small_fp64_matches_direct_sums(lp):
    w = workloads.rs_small(0)
    g = w["grid"]
    u0 = oracle.modulate(oracle.gaussian_beam(g, w["w0"]), w["phase"])
    with pytest.warns(lp.PropWarning):
        out = host(lp.rs_propagate(dev(u0, "c128"), g, w["wavelength"], w["z"]))
    ref = oracle.rs_propagate(u0, g, w["wavelength"], w["z"])
    e = rel_l2(out, ref)
    say("rs 128^2 fp64 rel-L2 vs oracle", e)
    assert e < 1e-12
    pix = [(0, 0), (127, 127), (64, 64), (3, 100), (90, 7)]
    direct = oracle.rs_at(u0, g, w["wavelength"], w["z"], pix)
    assert rel_l2(np.array([out[p] for p in pix]), direct) < 1e-12
    I = np.abs(out) ** 2
    assert rel_l2(I, np.abs(ref) ** 2) < 1e-12


RS_CASES = [
    (Grid(64, 64, 2e-6, 2e-6), 1, 600e-9, 200e-6),
    (Grid(100, 75, 1.5e-6, 2.5e-6, 3e-6, -2e-6), 2, 532e-9, 150e-6),
    (Grid(256, 256, 3e-6, 3e-6), 1, 650e-9, 2e-3),
    (Grid(1, 1, 1e-6, 1e-6), 3, 500e-9, 1e-5),
    (Grid(3, 200, 1e-6, 1e-6), 1, 500e-9, 1e-4),
    (Grid(384, 130, 2e-6, 2e-6), 1, 633e-9, 1e-3),
]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(RS_CASES)))
def test_rs_forward_and_adjoint(lp, kind, case):
    import warnings
    g, batch, wl, z = RS_CASES[case]
    say("rs case", case, kind, g, batch)
    u = cast(rnd((batch, g.ny, g.nx), case), kind)
    v = cast(rnd((batch, g.ny, g.nx), 100 + case), kind)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        out = host(lp.rs_propagate(dev(u, kind), g, wl, z))
        back = host(lp.rs_adjoint(dev(v, kind), g, wl, z))
    ef = rel_l2(out, oracle.rs_propagate(u, g, wl, z))
    ea = rel_l2(back, oracle.rs_adjoint(v, g, wl, z))
    say(f"  fwd {ef:.2e} adj {ea:.2e}")
    assert ef < TOL[kind] and ea < TOL[kind]


# ------------------------------------------------------------------ CZT --

CZT_CASES = [
    (Grid(64, 64, 2e-6, 2e-6), Grid(64, 64, 50e-9, 50e-9), 1, 600e-9, 5e-3),
    (Grid(90, 70, 3e-6, 2e-6, 1e-6, 2e-6), Grid(33, 41, 0.2e-6, 0.25e-6, -1e-6, 3e-6), 2, 532e-9, 2e-3),
    (Grid(256, 256, 4e-6, 4e-6), Grid(128, 128, 0.1e-6, 0.1e-6), 1, 650e-9, 25e-3),
    (Grid(1, 1, 1e-6, 1e-6), Grid(5, 3, 1e-6, 1e-6), 2, 500e-9, 1e-3),
    (Grid(300, 20, 2e-6, 2e-6), Grid(700, 9, 0.05e-6, 0.3e-6), 1, 700e-9, 1e-2),
]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(CZT_CASES)))
def test_czt_forward_and_adjoint(lp, kind, case):
    gi, win, batch, wl, z = CZT_CASES[case]
    say("czt case", case, kind)
    u = cast(rnd((batch, gi.ny, gi.nx), case), kind)
    v = cast(rnd((batch, win.ny, win.nx), 50 + case), kind)
    out = host(lp.czt_propagate(dev(u, kind), gi, win, wl, z))
    back = host(lp.czt_adjoint(dev(v, kind), gi, win, wl, z))
    ef = rel_l2(out, oracle.czt_propagate(u, gi, win, wl, z))
    ea = rel_l2(back, oracle.czt_adjoint(v, gi, win, wl, z))
    say(f"  fwd {ef:.2e} adj {ea:.2e}")
    assert ef < TOL[kind] and ea < TOL[kind]


# --------------------------------------------- headline shape, sampled --

def _pixels(n, seed, k=24):
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (n - 1, n - 1), (n // 2, n // 2), (0, n - 1)}
    while len(pts) < k:
        pts.add(tuple(int(v) for v in rng.integers(0, n, 2)))
    return sorted(pts)


def test_headline_2048_rs_czt_sampled(lp):
    """RS and CZT at 2048^2 (complex64) in the batched launch the benchmark
    times (batch 8), checked at sampled outputs by direct oracle sums.  Item
    k is item 0 times e^{0.1 i k}, so by linearity every item's output is
    item 0's times the same factor: that checks the indexing of all 8."""
    import torch
    w = workloads.rs_czt_2048(0)
    g, win, wl = w["grid"], w["window"], w["wavelength"]
    u0 = oracle.modulate(oracle.gaussian_beam(g, w["w0"], f=w["f"], wavelength=wl), w["phase"])
    u = cast(u0, "c64")
    ph = np.exp(0.1j * np.arange(8))
    du = dev(np.stack([u * p for p in ph]), "c64")

    def items_scale(out):
        # out[k] against out[0] e^{0.1 i k}, relative to |out[0]|
        ref = out[0]
        return max(rel_l2(out[k], ref * ph[k] / ph[0]) for k in range(1, 8))
    say("2048 rs forward")
    rs = host(lp.rs_propagate(du, g, wl, w["z_rs"]))
    pix = _pixels(2048, 1)
    ref = oracle.rs_at(u, g, wl, w["z_rs"], pix)
    e = rel_l2(np.array([rs[0][p] for p in pix]), ref)
    say("  rs sampled rel-L2", e)
    assert e < 1e-5
    es = items_scale(rs)
    say("  rs items vs item 0", es)
    assert es < 1e-5
    say("2048 rs adjoint")
    back = host(lp.rs_adjoint(torch.from_numpy(rs).to(torch.complex64).cuda(), g, wl, w["z_rs"]))
    refa = oracle.rs_adjoint_at(rs[0], g, wl, w["z_rs"], pix)
    e = rel_l2(np.array([back[0][p] for p in pix]), refa)
    say("  rs adjoint sampled rel-L2", e, "items vs item 0", items_scale(back))
    assert e < 1e-5 and items_scale(back) < 1e-5
    say("2048 czt forward")
    cz = host(lp.czt_propagate(du, g, win, wl, w["z_czt"]))
    refc = oracle.czt_at(u, g, win, wl, w["z_czt"], pix)
    e = rel_l2(np.array([cz[0][p] for p in pix]), refc)
    say("  czt sampled rel-L2", e, "items vs item 0", items_scale(cz))
    assert e < 1e-5 and items_scale(cz) < 1e-5
    say("2048 czt adjoint")
    cb = host(lp.czt_adjoint(torch.from_numpy(cz).to(torch.complex64).cuda(), g, win, wl, w["z_czt"]))
    refb = oracle.czt_adjoint_at(cz[0], g, win, wl, w["z_czt"], pix)
    e = rel_l2(np.array([cb[0][p] for p in pix]), refb)
    say("  czt adjoint sampled rel-L2", e, "items vs item 0", items_scale(cb))
    assert e < 1e-5 and items_scale(cb) < 1e-5


def test_repeat_launches_bitwise_identical(lp):
    g = Grid(200, 200, 2e-6, 2e-6)
    u = dev(rnd((2, 200, 200), 9), "c64")
    a = host(lp.rs_propagate(u, g, 600e-9, 1e-3))
    b = host(lp.rs_propagate(u, g, 600e-9, 1e-3))
    assert np.array_equal(a, b)
    win = Grid(50, 60, 0.1e-6, 0.1e-6)
    c = host(lp.czt_propagate(u, g, win, 600e-9, 1e-3))
    d = host(lp.czt_propagate(u, g, win, 600e-9, 1e-3))
    assert np.array_equal(c, d)


def test_nan_propagates(lp):
    g = Grid(32, 32, 2e-6, 2e-6)
    u = rnd((32, 32), 3)
    u[5, 7] = np.nan
    out = host(lp.rs_propagate(dev(u, "c64"), g, 600e-9, 1e-3))
    assert np.isnan(out).any()


def test_trace_all_passes_and_one_pass(lp):
    """The launch trace the benchmark reads: with every pass traced, an RS
    and a CZT call report their passes with launch counts, positive times
    and the algorithmic bytes of each launch; restricted to one pass, only
    that pass is reported; reading clears the trace."""
    import torch
    import warnings
    g = Grid.square(256, 1e-3)
    win = Grid.square(128, 20e-6)
    u = dev(rnd((2, 256, 256), 3), "c64")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        lp.rs_propagate(u, g, 600e-9, 5e-3)
        lp.czt_propagate(u, g, win, 600e-9, 5e-3)
        torch.cuda.synchronize()
        lp.prop_trace_enable(True)
        for _ in range(3):
            lp.rs_propagate(u, g, 600e-9, 5e-3)
            lp.czt_propagate(u, g, win, 600e-9, 5e-3)
        every = lp.prop_trace_read()
        lp.prop_trace_only("rs_cols")
        for _ in range(2):
            lp.rs_propagate(u, g, 600e-9, 5e-3)
            lp.czt_propagate(u, g, win, 600e-9, 5e-3)
        one = lp.prop_trace_read()
        empty = lp.prop_trace_read()
        lp.prop_trace_enable(False)
        lp.prop_trace_only(None)
    say("traced passes", {k: v[0] for k, v in every.items()}, "filtered", {k: v[0] for k, v in one.items()})
    assert {"rs_rows_fwd", "rs_cols", "rs_rows_inv", "czt_rows", "czt_cols"} <= set(every)
    assert all(v[0] == 3 and v[1] > 0 for k, v in every.items() if k.startswith(("rs_", "czt_")))
    # RS column pass: reads and writes the 256 x 512 workspace of each field, plus the spectrum once
    n, ms, by = every["rs_cols"]
    assert by / n >= 2 * 8 * 2 * 256 * 512
    assert set(one) == {"rs_cols"} and one["rs_cols"][0] == 2 and one["rs_cols"][1] > 0
    assert empty == {}
