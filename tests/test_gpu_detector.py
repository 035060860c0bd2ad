"""The paper's detector side on the GPU against the FP64 oracle: the
threshold-density loss (Methods, loss function), the STED effective
intensity (Methods, STED microscopy; worked values from the paper) and the
soft minimum over detectors (Methods, exploration of optical topologies)."""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads import Grid
from tests.conftest import rel_l2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sted_worked_examples.txt")


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


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _field(rng, shape, peak_at=None):
    # speckle-like field with a bright spot so that the threshold selects a region
    f = workloads.random_field(rng, shape)
    ny, nx = shape[-2:]
    yy, xx = np.mgrid[0:ny, 0:nx]
    cy, cx = peak_at or (ny // 3, nx // 2)
    return f * (0.3 + 3.0 * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / 40.0))


CASES = [("radial", 2, 0, 0.7), ("longitudinal", 1, 0, 0.5), ("sted", 2, 2, 0.7), ("sted_half", 2, 2, 0.3)]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_density_loss_vs_oracle(lp, kind, case):
    name, ncomp, ndep, eps = CASES[case]
    beta = 1.0 if name != "sted_half" else 0.4
    rng = np.random.default_rng(case + 10)
    b, ny, nx = 2, 37, 53
    comps = [cast(_field(rng, (b, ny, nx)), kind) for _ in range(ncomp)]
    dep = [cast(_field(rng, (b, ny, nx), (ny // 2, nx // 3)), kind) for _ in range(ndep)]
    res, gs, gd = lp.prop_density_loss([dev(c, kind) for c in comps], eps, [dev(d, kind) for d in dep] or None, beta)
    res = res.cpu().numpy()
    for bi in range(b):
        ref = oracle.density_loss_fields([c[bi] for c in comps], eps, [d[bi] for d in dep] or None, beta)
        loss, area, ieps, imax, seeds, seeds_dep = ref
        assert res[bi, 1] == area, (name, kind, res[bi], area)  # same FP64 intensities -> same selection
        assert abs(res[bi, 0] - loss) <= 1e-12 * loss and abs(res[bi, 2] - ieps) <= 1e-12 * ieps
        assert res[bi, 3] == imax or abs(res[bi, 3] - imax) <= 1e-15 * imax
        tol = 1e-6 if kind == "c64" else 1e-12
        for got, want in zip(gs + gd, seeds + seeds_dep):
            assert rel_l2(host(got)[bi], want) < tol
    say(f"density loss {name} {kind}: area {res[0, 1]:.0f} loss {res[0, 0]:.6e}")


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_sted_worked_examples_on_gpu(lp, kind):
    """Uniform beams with I_dep = ratio I_ex and eps = 0: every pixel is
    selected, so I_eps / (Area I_ex) is the printed effective fraction."""
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    closed = {"exp(-1/2)": math.exp(-0.5), "exp(-3/2)": math.exp(-1.5), "(1+exp(-1/2))/2": (1 + math.exp(-0.5)) / 2}
    a = 0.75 + 0.5j
    for beta, ratio, printed, form, dec in rows:
        ex = np.full((1, 8, 8), a)
        dep = np.full((1, 8, 8), a * math.sqrt(float(ratio)))
        res, _, _ = lp.prop_density_loss([dev(ex, kind)], 0.0, [dev(dep, kind)], float(beta), seeds=False)
        res = res.cpu().numpy()[0]
        i_ex = abs(complex(np.complex64(a) if kind == "c64" else a)) ** 2
        frac = res[2] / (res[1] * i_ex)
        say(f"  beta {beta} ratio {ratio}: I_eff/I_ex = {frac:.6f} (paper ~{printed}, {form})")
        assert res[1] == 64
        assert abs(frac - closed[form]) < (1e-6 if kind == "c64" else 1e-12)
        assert round(frac, int(dec)) == float(printed)


def test_softmin_vs_oracle(lp):
    import torch
    rng = np.random.default_rng(4)
    l = rng.uniform(0.1, 3.0, (5, 6))
    for beta in (0.5, 20.0):
        v, w = lp.prop_softmin(torch.from_numpy(l).cuda(), beta)
        for bi in range(5):
            rv, rw = oracle.softmin(l[bi], beta)
            assert abs(float(v[bi]) - rv) <= 1e-14 * max(1.0, abs(rv))
            assert np.abs(w[bi].cpu().numpy() - rw).max() <= 1e-14


def test_sted_focus_chain_gradient_fp64(lp):
    """STED setup of the paper in small: an excitation beam through an SLM
    and a depletion beam through a second SLM, both focused by the NA 0.9
    objective; loss = density loss (eps 0.7) of the STED effective radial
    intensity.  The autograd gradients with respect to both phase masks
    against the oracle's chain (FP64)."""
    import torch
    from paper_2310_08408_amd.autograd import VCZT, DensityLoss, Modulate
    n = 64
    g = Grid.square(n, 4e-3)
    win = Grid.square(40, 40 * 25e-9)
    wl, na = 532e-9, 0.9
    f = 2e-3 / na
    rng = np.random.default_rng(9)
    p1 = rng.uniform(-math.pi, math.pi, (1, n, n))
    p2 = rng.uniform(-math.pi, math.pi, (1, n, n))
    v = oracle.gaussian_beam(g, 1.2e-3) / math.sqrt(2.0)
    vt = dev(v[None], "c128")
    t1 = torch.tensor(p1, device="cuda", requires_grad=True)
    t2 = torch.tensor(p2, device="cuda", requires_grad=True)
    ex_x, ex_y = Modulate.apply(vt, t1), Modulate.apply(vt, t1)
    dp_x, dp_y = Modulate.apply(vt, t2), Modulate.apply(vt, t2)
    Ex = VCZT.apply(ex_x, ex_y, g, win, wl, 0.0, (na, f))
    Dx = VCZT.apply(dp_x, dp_y, g, win, wl, 0.0, (na, f))
    loss = DensityLoss.apply(2, 0.7, 1.0, Ex[0], Ex[1], Dx[0], Dx[1]).sum()
    loss.backward()
    # oracle chain
    u1, u2 = oracle.modulate(v, p1[0]), oracle.modulate(v, p2[0])
    E = oracle.vczt_focus(u1, u1, g, win, wl, na, f)
    D = oracle.vczt_focus(u2, u2, g, win, wl, na, f)
    L, area, _, _, s_ex, s_dep = oracle.density_loss_fields([E[0], E[1]], 0.7, [D[0], D[1]], 1.0)
    ga = oracle.vczt_focus_adjoint(s_ex[0], s_ex[1], np.zeros_like(s_ex[0]), g, win, wl, na, f)
    gd = oracle.vczt_focus_adjoint(s_dep[0], s_dep[1], np.zeros_like(s_dep[0]), g, win, wl, na, f)
    ref1 = oracle.phase_grad(ga[0], u1) + oracle.phase_grad(ga[1], u1)
    ref2 = oracle.phase_grad(gd[0], u2) + oracle.phase_grad(gd[1], u2)
    e_l = abs(float(loss) - L) / L
    e1 = rel_l2(t1.grad.cpu().numpy()[0], ref1)
    e2 = rel_l2(t2.grad.cpu().numpy()[0], ref2)
    say(f"STED chain: loss {float(loss):.6e} (oracle {L:.6e}, area {area:.0f}); grad rel-L2 {e1:.1e} {e2:.1e}")
    assert e_l < 1e-10 and e1 < 1e-9 and e2 < 1e-9
