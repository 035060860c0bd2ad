"""On-device optimiser step (Adam / AdamW, the optimisers of the paper's
Methods) against the oracle step, and a short discovery loop that drives an
SLM phase through the focusing chain on the GPU."""
import math
import sys
import warnings

import numpy as np
import pytest

import oracle
from workloads import Grid

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


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("wd", [0.0, 0.05])
def test_adam_step_vs_oracle(lp, dtype, wd):
    import torch
    dt = getattr(torch, dtype)
    rng = np.random.default_rng(12)
    n = 100003
    p0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) for _ in range(5)]
    if dtype == "float32":
        p0 = p0.astype(np.float32).astype(np.float64)
        grads = [g.astype(np.float32).astype(np.float64) for g in grads]
    p = torch.tensor(p0, dtype=dt, device="cuda")
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    rp, rm, rv = p0.copy(), np.zeros(n), np.zeros(n)
    for k, g in enumerate(grads, start=1):
        lp.prop_adam_step(p, torch.tensor(g, dtype=dt, device="cuda"), m, v, k, 0.02, weight_decay=wd)
        rp, rm, rv = oracle.adam_step(rp, g, rm, rv, k, 0.02, weight_decay=wd)
    err = np.abs(p.cpu().numpy().astype(np.float64) - rp).max() / np.abs(rp).max()
    say(f"adam {dtype} wd={wd}: max rel {err:.2e}")
    assert err < (1e-6 if dtype == "float32" else 1e-14)


def test_focus_discovery_loop(lp):
    """Radial beam -> SLM phase -> NA 0.9 objective -> spot size + E_z
    fraction: 40 device Adam steps on the phase lower the loss."""
    import torch
    from paper_2310_08408_amd.autograd import VCZT, Modulate, SpotLoss
    n = 96
    g = Grid.square(n, 4e-3)
    win = Grid.square(48, 48 * 40e-9)
    wl, na = 532e-9, 0.9
    f = 2e-3 / na
    vx, vy = lp.prop_source_radial(g, 1.2e-3)
    phi = torch.tensor(np.random.default_rng(3).uniform(-math.pi, math.pi, (1, n, n)), dtype=torch.float32,
                       device="cuda", requires_grad=True)
    opt = lp.Adam([phi], lr=0.05)
    losses = []
    for _ in range(40):
        opt.zero_grad()
        ux, uy = Modulate.apply(vx, phi), Modulate.apply(vy, phi)
        Ex, Ey, Ez = VCZT.apply(ux, uy, g, win, wl, 0.0, (na, f))
        loss = SpotLoss.apply(Ex, Ey, Ez, win, wl, 1.0).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    say(f"discovery loop: loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.8 * losses[0]
