"""GPU parity of the vectorial propagators (VRS, free-space VCZT, focusing
VCZT), the elementwise elements (sources, SLM, wave plate), the detector
loss and its seeds, against the FP64 oracle."""
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


def rnd(shape, seed):
    return workloads.random_field(np.random.default_rng(seed), shape)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def errs(got, ref):
    return max(rel_l2(g, r) for g, r in zip(got, ref))


VRS_CASES = [
    (Grid(48, 40, 2e-6, 2.5e-6, 1e-6, -1e-6), 1, 600e-9, 300e-6),
    (Grid(96, 96, 3e-6, 3e-6), 2, 532e-9, 2e-3),
    (Grid(1, 5, 1e-6, 1e-6), 1, 500e-9, 1e-5),
    # exact halves on schedules with the register hand-off (256 = 16*16,
    # 512 = 8*8*8): the complex64 mixing pass runs one 4-column tile per
    # workgroup with both transforms on the same threads
    (Grid(128, 128, 4e-6, 4e-6), 3, 633e-9, 4e-3),
    (Grid(256, 256, 2e-6, 2e-6, 0.5e-6, 0), 2, 532e-9, 1.5e-3),
    (Grid(1024, 1024, 4e-6, 4e-6), 1, 532e-9, 30e-3),      # 2048 = 16*8*16
]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(VRS_CASES)))
def test_vrs_forward_and_adjoint(lp, kind, case):
    import warnings
    g, b, wl, z = VRS_CASES[case]
    say("vrs", case, kind)
    ex, ey = (cast(rnd((b, g.ny, g.nx), s), kind) for s in (case, case + 10))
    gs = [cast(rnd((b, g.ny, g.nx), s), kind) for s in (20, 21, 22)]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        out = [host(t) for t in lp.vrs_propagate(dev(ex, kind), dev(ey, kind), g, wl, z)]
        back = [host(t) for t in lp.vrs_adjoint(*(dev(a, kind) for a in gs), g, wl, z)]
    ef = errs(out, oracle.vrs_propagate(ex, ey, g, wl, z))
    ea = errs(back, oracle.vrs_adjoint(*gs, g, wl, z))
    # FP64: the phase-conditioning bar of the FP64 RS kernel (derived in
    # test_gpu_edges.test_rs_full_4096_sampled): <= 3.5 eps k r between two
    # independent FP64 evaluations of k r (3.6e5 rad at 1024^2 over 30 mm)
    k_r = 2 * np.pi / wl * np.sqrt((g.nx * g.dx) ** 2 + (g.ny * g.dy) ** 2 + z * z)
    tol = TOL[kind] if kind == "c64" else max(TOL[kind], 3.5 * k_r * np.finfo(float).eps)
    say(f"  fwd {ef:.2e} adj {ea:.2e} (bar {tol:.1e})")
    assert ef < tol and ea < tol


VCZT_CASES = [
    (Grid(40, 36, 3e-6, 3e-6, 2e-6, 0), Grid(30, 26, 0.3e-6, 0.3e-6, 1e-6, -1e-6), 1, 600e-9, 1e-3),
    (Grid(128, 128, 4e-6, 4e-6), Grid(64, 64, 0.2e-6, 0.2e-6), 2, 650e-9, 5e-3),
]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(VCZT_CASES)))
def test_vczt_free_space(lp, kind, case):
    gi, win, b, wl, z = VCZT_CASES[case]
    say("vczt free", case, kind)
    ex, ey = (cast(rnd((b, gi.ny, gi.nx), s), kind) for s in (case, case + 3))
    gs = [cast(rnd((b, win.ny, win.nx), s), kind) for s in (30, 31, 32)]
    out = [host(t) for t in lp.vczt_propagate(dev(ex, kind), dev(ey, kind), gi, win, wl, z)]
    back = [host(t) for t in lp.vczt_adjoint(*(dev(a, kind) for a in gs), gi, win, wl, z)]
    ef = errs(out, oracle.vczt_propagate(ex, ey, gi, win, wl, z))
    ea = errs(back, oracle.vczt_adjoint(*gs, gi, win, wl, z))
    say(f"  fwd {ef:.2e} adj {ea:.2e}")
    assert ef < TOL[kind] and ea < TOL[kind]


FOCUS_CASES = [
    (Grid(64, 64, 4e-3 / 64, 4e-3 / 64), Grid(48, 40, 40e-9, 50e-9, 0.1e-6, 0), 1, 532e-9, 0.9),
    (Grid(127, 130, 3e-5, 3e-5), Grid(33, 33, 0.1e-6, 0.1e-6), 2, 635e-9, 0.6),
]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(FOCUS_CASES)))
def test_vczt_focus(lp, kind, case):
    gi, win, b, wl, na = FOCUS_CASES[case]
    f = (gi.nx * gi.dx / 2) / na
    say("vczt focus", case, kind)
    ex, ey = (cast(rnd((b, gi.ny, gi.nx), s), kind) for s in (case + 5, case + 6))
    gs = [cast(rnd((b, win.ny, win.nx), s), kind) for s in (40, 41, 42)]
    out = [host(t) for t in lp.vczt_propagate(dev(ex, kind), dev(ey, kind), gi, win, wl, lens=(na, f))]
    back = [host(t) for t in lp.vczt_adjoint(*(dev(a, kind) for a in gs), gi, win, wl, lens=(na, f))]
    ef = errs(out, oracle.vczt_focus(ex, ey, gi, win, wl, na, f))
    ea = errs(back, oracle.vczt_focus_adjoint(*gs, gi, win, wl, na, f))
    say(f"  fwd {ef:.2e} adj {ea:.2e}")
    assert ef < TOL[kind] and ea < TOL[kind]


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_sources_and_elements(lp, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    rdt = np.float32 if kind == "c64" else np.float64
    g = Grid(70, 50, 20e-6, 25e-6, 30e-6, -10e-6)
    wl = 650e-9
    src = host(lp.prop_source_gaussian(g, 300e-6, wl, amplitude=1.5, lens_f=25e-3, batch=2, dtype=dt))
    ref = oracle.gaussian_beam(g, 300e-6, 1.5, 25e-3, wl)
    assert rel_l2(src[1], ref) < TOL[kind]
    ex, ey = (host(t) for t in lp.prop_source_radial(g, 400e-6, dtype=dt))
    rx, ry = oracle.radial_beam(g, 400e-6)
    assert rel_l2(ex[0], rx) < TOL[kind] and rel_l2(ey[0], ry) < TOL[kind]
    v = cast(rnd((3, 50, 70), 1), kind)
    phi = np.random.default_rng(2).uniform(-math.pi, math.pi, (3, 50, 70)).astype(rdt)
    tphi = torch.from_numpy(phi).cuda()
    u = host(lp.prop_modulate(dev(v, kind), tphi))
    assert rel_l2(u, oracle.modulate(v, phi.astype(np.float64))) < TOL[kind]
    shared = host(lp.prop_modulate(dev(v, kind), tphi[:1].contiguous()))
    assert rel_l2(shared, oracle.modulate(v, phi[0].astype(np.float64))) < TOL[kind]
    gu = cast(rnd((3, 50, 70), 3), kind)
    gp = lp.prop_phase_grad(dev(gu, kind), dev(u, kind)).cpu().numpy()
    assert rel_l2(gp, oracle.phase_grad(gu, cast(u, kind))) < TOL[kind]
    # wave plate and its adjoint (parameter gradients reduced in FP64)
    gx, gy = cast(rnd((2, 50, 70), 4), kind), cast(rnd((2, 50, 70), 5), kind)
    a, b = cast(rnd((2, 50, 70), 6), kind), cast(rnd((2, 50, 70), 7), kind)
    ox, oy = (host(t) for t in lp.prop_waveplate(dev(a, kind), dev(b, kind), 0.7, -0.4))
    rx, ry = oracle.waveplate(a, b, 0.7, -0.4)
    assert rel_l2(ox, rx) < TOL[kind] and rel_l2(oy, ry) < TOL[kind]
    gex, gey, dp = lp.prop_waveplate_adjoint(dev(gx, kind), dev(gy, kind), dev(a, kind), dev(b, kind), 0.7, -0.4)
    for bi in range(2):
        rgx, rgy, de, dth = oracle.waveplate_adjoint(gx[bi], gy[bi], a[bi], b[bi], 0.7, -0.4)
        assert rel_l2(host(gex)[bi], rgx) < TOL[kind]
        assert rel_l2(host(gey)[bi], rgy) < TOL[kind]
        d = dp.cpu().numpy()[bi]
        tol = 1e-5 if kind == "c64" else 1e-11
        assert abs(d[0] - de) <= tol * max(1, abs(de)) and abs(d[1] - dth) <= tol * max(1, abs(dth))


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("with_ez", [False, True])
def test_spot_loss_and_seeds(lp, kind, with_ez):
    win = Grid(40, 32, 25e-9, 30e-9, 0.2e-6, -0.1e-6)
    E = [cast(rnd((2, 32, 40), s), kind) for s in (11, 12, 13)]
    wl, wfz = 532e-9, (0.8 if with_ez else 0.0)
    res, seeds = lp.prop_spot_loss(dev(E[0], kind), dev(E[1], kind), dev(E[2], kind) if with_ez else None, win, wl,
                                   wfz)
    res = res.cpu().numpy()
    for b in range(2):
        loss, s2, fz, ref_seeds = oracle.spot_loss(win, wl, E[0][b], E[1][b], E[2][b] if with_ez else None, wfz)
        tol = 1e-5 if kind == "c64" else 1e-11
        assert abs(res[b, 0] - loss) <= tol * abs(loss)
        assert abs(res[b, 1] - s2) <= tol * abs(s2)
        assert abs(res[b, 2] - fz) <= tol * max(abs(fz), 1e-30) + (tol if with_ez else 0)
        for c in range(3 if with_ez else 2):
            assert rel_l2(host(seeds[c])[b], ref_seeds[c]) < (1e-5 if kind == "c64" else 1e-10)


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_vector_config_2048_sampled(lp, kind):
    """The vectorial workload at full size (2048^2, 4 mm grid, 532 nm): VRS
    over 50 mm and the NA 0.9 objective (f = 2.222 mm) onto a 4 um window,
    forward and adjoint, at sampled outputs against the oracle's direct
    sums.  FP64 bar for VRS: each side rounds the kernel phase k r (up to
    6e5 rad here) by about k r eps."""
    import torch
    import warnings
    n = 2048
    g = Grid.square(n, 4e-3)
    win = Grid.square(n, 4e-6)
    wl, z, na = 532e-9, 50e-3, 0.9
    f = (n * g.dx / 2) / na
    rng = np.random.default_rng(17)
    ex, ey = (cast(rnd((1, n, n), s), kind) for s in (71, 72))
    gs = [cast(rnd((1, n, n), s), kind) for s in (73, 74, 75)]
    pix = [(0, 0), (n - 1, n - 1), (n // 2, n // 2), (5, n - 9), (1500, 40)]
    pix += [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(3)]
    # pupil pixels for the focus adjoint: inside the aperture (the corners lie outside)
    pin = [(n // 2, n // 2), (n // 2 + 300, n // 2 - 700), (400, 1100), (1700, 900), (n // 2, 60)]
    say(f"2048 vrs forward/adjoint {kind}")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        vf = [host(t)[0] for t in lp.vrs_propagate(dev(ex, kind), dev(ey, kind), g, wl, z)]
        vb = [host(t)[0] for t in lp.vrs_adjoint(*(dev(a, kind) for a in gs), g, wl, z)]
    rf = oracle.vrs_at(ex[0], ey[0], g, wl, z, pix)
    rb = oracle.vrs_adjoint_at(gs[0][0], gs[1][0], gs[2][0], g, wl, z, pix)
    e_vf = max(rel_l2(np.array([vf[c][p] for p in pix]), rf[c]) for c in range(3))
    e_vb = max(rel_l2(np.array([vb[c][p] for p in pix]), rb[c]) for c in range(2))
    say(f"  vrs sampled rel-L2: fwd {e_vf:.2e} adj {e_vb:.2e}")
    say("2048 focus forward/adjoint")
    ff = [host(t)[0] for t in lp.vczt_propagate(dev(ex, kind), dev(ey, kind), g, win, wl, lens=(na, f))]
    fb = [host(t)[0] for t in lp.vczt_adjoint(*(dev(a, kind) for a in gs), g, win, wl, lens=(na, f))]
    torch.cuda.synchronize()
    qf = oracle.vczt_focus_at(ex[0], ey[0], g, win, wl, na, f, pix)
    qb = oracle.vczt_focus_adjoint_at(gs[0][0], gs[1][0], gs[2][0], g, win, wl, na, f, pin)
    e_ff = max(rel_l2(np.array([ff[c][p] for p in pix]), qf[c]) for c in range(3))
    e_fb = max(rel_l2(np.array([fb[c][p] for p in pin]), qb[c]) for c in range(2))
    say(f"  focus sampled rel-L2: fwd {e_ff:.2e} adj {e_fb:.2e}")
    if kind == "c64":
        assert max(e_vf, e_vb, e_ff, e_fb) < TOL["c64"]
    else:
        # the phase-conditioning bar of the FP64 RS kernel (derived in
        # test_gpu_edges.test_rs_full_4096_sampled): <= 3.5 eps k r between two
        # independent FP64 evaluations of k r
        k_r = 2 * np.pi / wl * np.hypot(np.hypot(n * g.dx, n * g.dy), z)
        assert max(e_vf, e_vb) < 3.5 * k_r * np.finfo(float).eps and max(e_ff, e_fb) < TOL["c128"]
