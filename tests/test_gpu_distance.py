"""Distance gradients dL/dz of RS and CZT on the GPU against the FP64 oracle
(every setup of the paper optimises its distances together with the phase
masks: Results; Methods, parameter spaces with distances z_i)."""
import math
import sys
import warnings

import numpy as np
import pytest

import oracle
import workloads
from workloads import Grid

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-4, "c128": 1e-10}


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    return lp


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def cast(a, kind):
    return np.asarray(a, np.complex64 if kind == "c64" else np.complex128).astype(np.complex128)


def rnd(shape, seed):
    return workloads.random_field(np.random.default_rng(seed), shape)


RS_CASES = [(Grid(40, 36, 3e-6, 4e-6, 1e-6, 0), 2, 600e-9, 400e-6), (Grid(96, 130, 2e-6, 2e-6), 1, 532e-9, 1e-3)]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(RS_CASES)))
def test_rs_grad_z(lp, kind, case):
    g, b, wl, z = RS_CASES[case]
    u = cast(rnd((b, g.ny, g.nx), case + 1), kind)
    c = cast(rnd((b, g.ny, g.nx), case + 50), kind)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        got = lp.rs_grad_z(dev(u, kind), dev(c, kind), g, wl, z).cpu().numpy()
    ref = np.atleast_1d(oracle.rs_grad_z(u, c, g, wl, z))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"rs_grad_z case {case} {kind}: rel {err:.2e}")
    assert err < TOL[kind]


FUSED_CASES = RS_CASES + [(Grid(37, 5, 3e-6, 2e-6, 0, 1e-6), 3, 600e-9, 300e-6),
                          (Grid(1, 24, 2e-6, 2e-6), 2, 532e-9, 200e-6)]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(FUSED_CASES)))
def test_rs_adjoint_grad_z_matches_separate_calls(lp, kind, case):
    """rs_adjoint_grad_z: its field gradient bit-identical to rs_adjoint, its
    dz within rounding of rs_grad_z (the sum taken in the row-spectrum
    domain) and of the oracle.  Cases: ragged grids, batch 1-3, and nx = 1
    (padded workspace rows: the two computations run separately)."""
    import torch
    g, b, wl, z = FUSED_CASES[case]
    u = cast(rnd((b, g.ny, g.nx), case + 7), kind)
    c = cast(rnd((b, g.ny, g.nx), case + 70), kind)
    ut, ct = dev(u, kind), dev(c, kind)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gu, dz = lp.rs_adjoint_grad_z(ct, ut, g, wl, z)
        gu_ref = lp.rs_adjoint(ct, g, wl, z)
        dz_ref = lp.rs_grad_z(ut, ct, g, wl, z).cpu().numpy()
        with pytest.raises(lp.PropError):
            lp.rs_adjoint_grad_z(ct, ut, g, wl, z, out=ct)
    assert torch.equal(gu, gu_ref)
    dz = dz.cpu().numpy()
    ref = np.atleast_1d(oracle.rs_grad_z(u, c, g, wl, z))
    e_sep = np.abs(dz - dz_ref).max() / np.abs(dz_ref).max()
    e_orc = np.abs(dz - ref).max() / np.abs(ref).max()
    say(f"rs_adjoint_grad_z case {case} {kind}: dz vs rs_grad_z {e_sep:.2e}, vs oracle {e_orc:.2e}")
    assert e_sep < TOL[kind] and e_orc < TOL[kind]


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_rs_adjoint_grad_z_1024_batch4(lp, kind):
    """The lattice's shape (1024^2 grid, 4 planes): against the separate
    calls (the oracle at this size is covered by the 2048^2 test of
    rs_grad_z)."""
    import torch
    g, wl, z = Grid.square(1024, 1024 * 4.8e-6), 532e-9, 0.03
    gen = torch.Generator(device="cuda").manual_seed(3)
    dt = torch.complex64 if kind == "c64" else torch.complex128
    u = torch.randn((4, 1024, 1024), dtype=dt, device="cuda", generator=gen)
    c = torch.randn((4, 1024, 1024), dtype=dt, device="cuda", generator=gen)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gu, dz = lp.rs_adjoint_grad_z(c, u, g, wl, z)
        gu_ref = lp.rs_adjoint(c, g, wl, z)
        dz_ref = lp.rs_grad_z(u, c, g, wl, z)
    assert torch.equal(gu, gu_ref)
    err = float((dz - dz_ref).abs().max() / dz_ref.abs().max())
    say(f"rs_adjoint_grad_z 1024^2 x4 {kind}: dz vs rs_grad_z {err:.2e}")
    assert err < TOL[kind]


CZT_CASES = [(Grid(40, 36, 3e-6, 3e-6, 2e-6, 0), Grid(30, 26, 0.3e-6, 0.3e-6, 1e-6, -1e-6), 2, 600e-9, 1e-3),
             (Grid(128, 96, 4e-6, 4e-6), Grid(64, 80, 0.2e-6, 0.25e-6), 1, 650e-9, 5e-3)]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(CZT_CASES)))
@pytest.mark.parametrize("give_u_out", [False, True])
def test_czt_grad_z(lp, kind, case, give_u_out):
    gi, win, b, wl, z = CZT_CASES[case]
    u = cast(rnd((b, gi.ny, gi.nx), case + 3), kind)
    c = cast(rnd((b, win.ny, win.nx), case + 60), kind)
    ud = dev(u, kind)
    uo = lp.czt_propagate(ud, gi, win, wl, z) if give_u_out else None
    got = lp.czt_grad_z(ud, dev(c, kind), gi, win, wl, z, u_out=uo).cpu().numpy()
    ref = np.atleast_1d(oracle.czt_grad_z(u, c, gi, win, wl, z))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"czt_grad_z case {case} {kind} u_out={give_u_out}: rel {err:.2e}")
    assert err < TOL[kind]


def test_distance_gradients_through_autograd_fp64(lp):
    """SLM -> RS(z1) -> CZT(z2) -> |U|^2 loss: dL/dz1, dL/dz2 from the
    autograd chain against central differences of the FP64 GPU forward."""
    import torch
    from paper_2310_08408_amd.autograd import CZT, RS, Modulate
    g = Grid(48, 40, 10e-6, 10e-6)
    win = Grid(24, 20, 2e-6, 2e-6)
    wl = 600e-9
    v = lp.prop_source_gaussian(g, 150e-6, wl, dtype=torch.complex128)
    phi = torch.tensor(np.random.default_rng(5).uniform(-1, 1, (1, 40, 48)), device="cuda")

    def loss(z1, z2):
        u = Modulate.apply(v, phi)
        y = RS.apply(u, g, wl, z1)
        w = CZT.apply(y, g, win, wl, z2)
        return (w.abs() ** 2).sum()

    z1 = torch.tensor(3e-3, dtype=torch.float64, device="cuda", requires_grad=True)
    z2 = torch.tensor(8e-3, dtype=torch.float64, device="cuda", requires_grad=True)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        L = loss(z1, z2)
        L.backward()
        with torch.no_grad():
            # central differences at h and h/2, Richardson-extrapolated (the
            # loss is a large sum, so h must not be too small either)
            def cd(f, h):
                return (f(h) - f(-h)) / (2 * h)

            def rich(f, h=2e-9):
                return (4 * cd(f, h / 2) - cd(f, h)) / 3

            fd1 = rich(lambda d: float(loss(3e-3 + d, 8e-3)))
            fd2 = rich(lambda d: float(loss(3e-3, 8e-3 + d)))
    # the oracle's analytic chain (same inputs, FP64)
    u = oracle.modulate(oracle.gaussian_beam(g, 150e-6), phi.cpu().numpy()[0])
    y = oracle.rs_propagate(u, g, wl, 3e-3)
    w = oracle.czt_propagate(y, g, win, wl, 8e-3)
    ref2 = oracle.czt_grad_z(y, 2 * w, g, win, wl, 8e-3)
    ref1 = oracle.rs_grad_z(u, oracle.czt_adjoint(2 * w, g, win, wl, 8e-3), g, wl, 3e-3)
    d1, d2 = float(z1.grad), float(z2.grad)
    say(f"autograd dz1 {d1:.9e} oracle {ref1:.9e} FD {fd1:.6e}; dz2 {d2:.9e} oracle {ref2:.9e} FD {fd2:.6e}")
    assert abs(d1 - ref1) <= 1e-9 * abs(ref1) and abs(d2 - ref2) <= 1e-9 * abs(ref2)
    assert abs(d1 - fd1) <= 1e-4 * abs(fd1) and abs(d2 - fd2) <= 1e-4 * abs(fd2)


def test_distance_gradients_2048(lp):
    """Headline geometry (2048^2 on 4 mm, 650 nm; RS z = 25 mm, CZT z = f onto
    40 um): FP32 dL/dz against the FP64 GPU path for a batch of 2, and item
    0 of both against the FP64 oracle."""
    import torch
    w = workloads.rs_czt_2048(0)
    g, win, wl = w["grid"], w["window"], w["wavelength"]
    u64 = oracle.modulate(oracle.gaussian_beam(g, w["w0"], f=w["f"], wavelength=wl), w["phase"])
    u64 = u64.astype(np.complex64).astype(np.complex128)
    c64 = workloads.random_field(np.random.default_rng(7), (g.ny, g.nx)).astype(np.complex64).astype(np.complex128)
    cw = workloads.random_field(np.random.default_rng(8), (win.ny, win.nx)).astype(np.complex64).astype(np.complex128)
    res = {}
    for kind in ("c64", "c128"):
        u = dev(np.stack([u64, 0.5 * u64]), kind)
        gr = dev(np.stack([c64, c64]), kind)
        gc = dev(np.stack([cw, cw]), kind)
        res[kind] = (lp.rs_grad_z(u, gr, g, wl, w["z_rs"]).cpu().numpy(),
                     lp.czt_grad_z(u, gc, g, win, wl, w["z_czt"]).cpu().numpy())
    e_rs = np.abs(res["c64"][0] - res["c128"][0]).max() / np.abs(res["c128"][0]).max()
    e_czt = np.abs(res["c64"][1] - res["c128"][1]).max() / np.abs(res["c128"][1]).max()
    say(f"2048: fp32 vs fp64 rel: rs {e_rs:.2e} czt {e_czt:.2e}")
    assert e_rs < 1e-4 and e_czt < 1e-4
    ref_rs = oracle.rs_grad_z(u64, c64, g, wl, w["z_rs"])
    ref_czt = oracle.czt_grad_z(u64, cw, g, win, wl, w["z_czt"])
    for kind, tol in (("c64", 1e-4), ("c128", 1e-9)):
        er = abs(res[kind][0][0] - ref_rs) / abs(ref_rs)
        ec = abs(res[kind][1][0] - ref_czt) / abs(ref_czt)
        say(f"  {kind} vs oracle: rs {er:.2e} czt {ec:.2e}")
        assert er < tol and ec < tol
