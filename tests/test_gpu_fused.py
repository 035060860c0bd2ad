"""Adjoints fused with the SLM phase gradient (the adjoint's last pass writes
Im(g_U conj U) directly) against the unfused library calls and the FP64
oracle (paper: Methods, the per-pixel SLM phases and their gradients)."""
import sys
import warnings

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


def dev(a, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def cast(a, kind):
    return np.asarray(a, np.complex64 if kind == "c64" else np.complex128).astype(np.complex128)


TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("accumulate", [False, True])
def test_rs_adjoint_phase_grad(lp, kind, accumulate):
    import torch
    g = Grid(70, 45, 3e-6, 4e-6, 1e-6, 0)
    wl, z = 600e-9, 300e-6
    rng = np.random.default_rng(3)
    u = cast(workloads.random_field(rng, (2, 45, 70)), kind)
    go = cast(workloads.random_field(rng, (2, 45, 70)), kind)
    base = rng.standard_normal((2, 45, 70))
    rdt = torch.float32 if kind == "c64" else torch.float64
    grad = torch.tensor(base, dtype=rdt, device="cuda")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        grad, gu = lp.rs_adjoint_phase_grad(dev(go, kind), dev(u, kind), g, wl, z, grad=grad, accumulate=accumulate,
                                            g_u=True)
        ref_gu = lp.rs_adjoint(dev(go, kind), g, wl, z)
    ref = oracle.phase_grad(oracle.rs_adjoint(go, g, wl, z), u) + (base if accumulate else 0)
    e_grad = rel_l2(grad.cpu().numpy(), ref)
    e_gu = rel_l2(gu.cpu().numpy(), ref_gu.cpu().numpy())
    say(f"rs fused {kind} acc={accumulate}: grad vs oracle {e_grad:.2e}, g_U vs unfused {e_gu:.2e}")
    assert e_grad < TOL[kind] and e_gu < (1e-6 if kind == "c64" else 1e-13)


CZT_CASES = [(Grid(64, 48, 3e-6, 3e-6, 2e-6, 0), Grid(40, 30, 0.3e-6, 0.3e-6, 1e-6, -1e-6)),
             (Grid(96, 96, 4e-6, 4e-6), Grid(96, 96, 0.2e-6, 0.2e-6))]


@pytest.mark.parametrize("kind", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(CZT_CASES)))
def test_czt_adjoint_phase_grad(lp, kind, case):
    gi, win = CZT_CASES[case]
    wl, z = 650e-9, 4e-3
    rng = np.random.default_rng(case + 20)
    u = cast(workloads.random_field(rng, (2, gi.ny, gi.nx)), kind)
    go = cast(workloads.random_field(rng, (2, win.ny, win.nx)), kind)
    grad, gu = lp.czt_adjoint_phase_grad(dev(go, kind), dev(u, kind), gi, win, wl, z, g_u=True)
    ref_g = oracle.czt_adjoint(go, gi, win, wl, z)
    e_grad = rel_l2(grad.cpu().numpy(), oracle.phase_grad(ref_g, u))
    e_gu = rel_l2(gu.cpu().numpy(), ref_g)
    grad2, none = lp.czt_adjoint_phase_grad(dev(go, kind), dev(u, kind), gi, win, wl, z)
    assert none is None
    say(f"czt fused {kind} case {case}: grad {e_grad:.2e} g_U {e_gu:.2e}")
    assert e_grad < TOL[kind] and e_gu < TOL[kind]
    assert rel_l2(grad2.cpu().numpy(), grad.cpu().numpy()) < 1e-15
