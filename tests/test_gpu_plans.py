"""Batched uneven setups through the plan API (one graph launch per
direction): every setup's results equal the single calls and the FP64 oracle
(paper: Results, batches of candidate setups evaluated per step)."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import Grid
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu


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


def _uneven(seed, count, sizes):
    return list(workloads.uneven_96(seed, count=count, sizes=sizes))


@pytest.mark.parametrize("graph", [False, True])
def test_uneven_rs_lens_czt_plans(lp, graph):
    """Uneven setups: SLM phase -> RS(z) [plan A], thin lens f -> CZT at z = f
    onto a small window [plan B]; forward then adjoint, graph or eager."""
    import torch
    import warnings
    setups = _uneven(3, 6, (48, 64, 96, 130))
    ta, tb, keep = [], [], []
    for w in setups:
        g = w["grid"]
        n = g.nx
        win = Grid.square(40, 40 * 0.5e-6)
        v = lp.prop_source_gaussian(g, 0.6e-3, w["wavelength"])
        phi = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda")
        a = torch.empty_like(v)
        y = torch.empty((1, 40, 40), dtype=torch.complex64, device="cuda")
        gy = torch.randn_like(y)
        ga, gv = torch.empty_like(v), torch.empty_like(v)
        gphi = torch.empty_like(phi)
        ta.append(lp.Setup(lp.PROP_OP_RS, g, [v], [a], [ga], w["wavelength"], w["z"], phase=phi, grad_inputs=[gv],
                           grad_phase=gphi))
        tb.append(lp.Setup(lp.PROP_OP_CZT, g, [a], [y], [gy], w["wavelength"], w["f"], window=win, lens_f=w["f"],
                           grad_inputs=[ga]))
        keep.append((w, v, phi, a, y, gy, ga, gv, gphi, win))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        pa, pb = lp.Plan(ta, graph=graph), lp.Plan(tb, graph=graph)
        for rep in range(2):  # replays must agree
            pa.forward(); pb.forward(); pb.adjoint(); pa.adjoint()
            torch.cuda.synchronize()
            for i, (w, v, phi, a, y, gy, ga, gv, gphi, win) in enumerate(keep):
                g, wl = w["grid"], w["wavelength"]
                u = lp.prop_modulate(v, phi)
                ref_a = lp.rs_propagate(u, g, wl, w["z"])
                assert rel_l2(a.cpu().numpy(), ref_a.cpu().numpy()) < 1e-6
                # oracle on the same (cast) inputs
                u64 = u.cpu().numpy().astype(np.complex128)[0]
                ra = oracle.rs_propagate(u64, g, wl, w["z"])
                assert rel_l2(a.cpu().numpy()[0], ra) < 1e-5
                a64 = a.cpu().numpy().astype(np.complex128)[0]
                lensed = a64 * np.exp(-1j * (2 * math.pi / wl) * (oracle.coords(g)[0][None, :] ** 2 +
                                                                 oracle.coords(g)[1][:, None] ** 2) / (2 * w["f"]))
                ry = oracle.czt_propagate(lensed, g, win, wl, w["f"])
                assert rel_l2(y.cpu().numpy()[0], ry) < 1e-5
                # adjoint chain against the oracle
                gy64 = gy.cpu().numpy().astype(np.complex128)[0]
                g_lensed = oracle.czt_adjoint(gy64, g, win, wl, w["f"])
                lens_conj = np.exp(1j * (2 * math.pi / wl) * (oracle.coords(g)[0][None, :] ** 2 +
                                                           oracle.coords(g)[1][:, None] ** 2) / (2 * w["f"]))
                rga = g_lensed * lens_conj
                assert rel_l2(ga.cpu().numpy()[0], rga) < 1e-5
                ga64 = ga.cpu().numpy().astype(np.complex128)[0]
                gu = oracle.rs_adjoint(ga64, g, wl, w["z"])
                rgphi = oracle.phase_grad(gu, u64)
                assert rel_l2(gphi.cpu().numpy()[0], rgphi) < 1e-4
                rgv = gu * np.exp(-1j * phi.cpu().numpy().astype(np.float64)[0])
                assert rel_l2(gv.cpu().numpy()[0], rgv) < 1e-5
            say(f"graph={graph} replay {rep}: {len(keep)} setups agree with single calls and the oracle")
    pa.close(); pb.close()


def test_vector_plan_matches_single_calls(lp):
    import torch
    g = Grid(64, 48, 3e-5, 3e-5)
    win = Grid(32, 32, 0.1e-6, 0.1e-6)
    ex, ey = (torch.randn((1, 48, 64), dtype=torch.complex128, device="cuda") for _ in range(2))
    outs = [torch.empty((1, 32, 32), dtype=torch.complex128, device="cuda") for _ in range(3)]
    gouts = [torch.randn((1, 32, 32), dtype=torch.complex128, device="cuda") for _ in range(3)]
    gins = [torch.empty_like(ex) for _ in range(2)]
    vr = [torch.empty_like(ex) for _ in range(3)]
    gvr = [torch.randn_like(ex) for _ in range(3)]
    gvin = [torch.empty_like(ex) for _ in range(2)]
    phi = torch.rand((1, 48, 64), dtype=torch.float64, device="cuda")
    gphi = torch.empty_like(phi)
    na, f = 0.8, (64 * 3e-5 / 2) / 0.8
    s1 = lp.Setup(lp.PROP_OP_VCZT, g, [ex, ey], outs, gouts, 532e-9, window=win, lens=(na, f), phase=phi,
                  grad_inputs=gins, grad_phase=gphi)
    s2 = lp.Setup(lp.PROP_OP_VRS, g, [ex, ey], vr, gvr, 532e-9, 2e-3, grad_inputs=gvin)
    p = lp.Plan([s1, s2], dtype=torch.complex128, graph=True)
    p.forward(); p.adjoint()
    torch.cuda.synchronize()
    ux, uy = lp.prop_modulate(ex, phi), lp.prop_modulate(ey, phi)
    ref = lp.vczt_propagate(ux, uy, g, win, 532e-9, lens=(na, f))
    for a, b in zip(outs, ref):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-13
    gux, guy = lp.vczt_adjoint(*gouts, g, win, 532e-9, lens=(na, f))
    rg = lp.prop_phase_grad(gux, ux) + lp.prop_phase_grad(guy, uy)
    assert rel_l2(gphi.cpu().numpy(), rg.cpu().numpy()) < 1e-12
    assert rel_l2(gins[0].cpu().numpy(), lp.prop_modulate(gux, -phi).cpu().numpy()) < 1e-13
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        rv = lp.vrs_propagate(ex, ey, g, 532e-9, 2e-3)
        rgv = lp.vrs_adjoint(*gvr, g, 532e-9, 2e-3)
    for a, b in zip(vr, rv):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-13
    for a, b in zip(gvin, rgv):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-13
    p.close()


def test_plan_rejects_bad_setups(lp):
    import torch
    g = Grid(16, 16, 1e-6, 1e-6)
    v = torch.zeros((1, 16, 16), dtype=torch.complex64, device="cuda")
    bad = lp.Setup(lp.PROP_OP_RS, g, [v], [v.clone()], [v.clone()], -1.0, 1e-3)
    with pytest.raises(lp.PropError):
        lp.Plan([bad])
