"""The allocation-free detector loss (prop_spot_loss_noalloc) against the
allocating entry point, through the C ABI: two calls in a row, the second
smaller, then a batch beyond its fixed scratch."""
import numpy as np
import pytest

import workloads
from workloads import Grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    return lp


def _fields(rng, batch, win, dt):
    import torch
    return [torch.from_numpy(workloads.random_field(rng, (batch, win.ny, win.nx))).to(dt).cuda() for _ in range(3)]


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_noalloc_spot_loss_matches_allocating_entry(lp, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    rng = np.random.default_rng(21)
    for batch, win, wfz, with_ez in ((5, Grid(200, 160, 2e-9, 2.5e-9, 1e-8, -2e-8), 0.3, True),
                                     (2, Grid(64, 48, 3e-9, 3e-9), 0.0, False)):
        ex, ey, ez = _fields(rng, batch, win, dt)
        ez = ez if with_ez else None
        r0, s0 = lp.prop_spot_loss(ex, ey, ez, win, 532e-9, wfz)
        r1, s1 = lp.prop_spot_loss(ex, ey, ez, win, 532e-9, wfz, noalloc=True)
        torch.cuda.synchronize()
        # same kernels and reduction order: identical numbers
        assert torch.equal(r0, r1), (batch, (r0 - r1).abs().max())
        for a, b in zip(s0, s1):
            if a is not None:
                assert torch.equal(a, b)
        assert bool(torch.isfinite(r1).all())


def test_noalloc_spot_loss_limit(lp):
    import torch
    win = Grid(8, 8, 1e-9, 1e-9)
    ex = torch.ones((257, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(lp.PropError) as e:
        lp.prop_spot_loss(ex, ex.clone(), None, win, 532e-9, noalloc=True, seeds=False)
    assert e.value.status == -7
    r, _ = lp.prop_spot_loss(ex[:256], ex[:256].clone(), None, win, 532e-9, noalloc=True, seeds=False)
    torch.cuda.synchronize()
    assert r.shape == (256, 8)
