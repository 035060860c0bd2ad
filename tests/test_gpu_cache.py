"""Lifetime of the library's cached tables on the GPU: plans pin what their
kernels and graphs address, the byte budget bounds the cache under distance
optimisation (every experiment of the paper optimises distances: Results;
Methods, the large-scale search space), tables generated on one stream are
waited for on another, and a forced allocation failure leaves the caller's
buffers untouched."""
import math
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
    yield lp
    lp.prop_cache_set_limit(0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _small_plan(lp, torch, graph, seed):
    rng = np.random.default_rng(seed)
    g = Grid.square(96, 96 * 8e-6)
    win = Grid.square(40, 40 * 0.4e-6)
    u = torch.from_numpy(workloads.random_field(rng, (2, 96, 96)).astype(np.complex64)).cuda()
    gy = torch.from_numpy(workloads.random_field(rng, (2, 40, 40)).astype(np.complex64)).cuda()
    y_rs, g_rs = torch.empty_like(u), torch.empty_like(u)
    y_czt, g_czt = torch.empty_like(gy), torch.empty_like(u)
    s1 = lp.Setup(lp.PROP_OP_RS, g, [u], [y_rs], [y_rs], 600e-9, 31e-3 + seed * 1e-6, grad_inputs=[g_rs])
    s2 = lp.Setup(lp.PROP_OP_CZT, g, [u], [y_czt], [gy], 600e-9, 47e-3 + seed * 1e-6, window=win,
                  grad_inputs=[g_czt])
    return lp.Plan([s1, s2], graph=graph), (g, win, u, gy, y_rs, g_rs, y_czt, g_czt, 31e-3 + seed * 1e-6,
                                            47e-3 + seed * 1e-6)


@pytest.mark.parametrize("graph", [True, False])
def test_plan_survives_cache_clear(lp, graph):
    """prop_cache_clear while a plan lives: the plan's pinned spectra, zoom
    vectors and twiddles stay, so a replay (graph) or an eager run reads
    valid tables and matches the single calls; after destroy they are
    ordinary cache entries again."""
    import torch
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        plan, (g, win, u, gy, y_rs, g_rs, y_czt, g_czt, z1, z2) = _small_plan(lp, torch, graph, 3 if graph else 4)
        info = lp.prop_cache_info()
        assert info["pinned"] >= 4, info   # two twiddle lengths, one spectrum, zoom vectors
        plan.forward(); plan.adjoint()
        torch.cuda.synchronize()
        first = [host(t) for t in (y_rs, g_rs, y_czt, g_czt)]
        lp.prop_cache_clear()
        after = lp.prop_cache_info()
        assert after["pinned"] == info["pinned"] and after["spectra"] >= 1
        for t in (y_rs, g_rs, y_czt, g_czt):
            t.zero_()
        plan.forward(); plan.adjoint()
        torch.cuda.synchronize()
        second = [host(t) for t in (y_rs, g_rs, y_czt, g_czt)]
        for a, b in zip(first, second):
            assert np.array_equal(a, b)
        ref = [lp.rs_propagate(u, g, 600e-9, z1), lp.rs_adjoint(y_rs, g, 600e-9, z1),
               lp.czt_propagate(u, g, win, 600e-9, z2), lp.czt_adjoint(gy, g, win, 600e-9, z2)]
        for a, b in zip(second, ref):
            assert rel_l2(a, host(b)) < 1e-6
        plan.close()
    assert lp.prop_cache_info()["pinned"] == 0
    lp.prop_cache_clear()


def test_lru_budget_and_recompute(lp):
    """With a small budget, RS at many distances evicts old spectra (in
    rounds, one device synchronisation each); a distance whose spectrum was
    evicted is recomputed and gives the same field bit for bit."""
    import torch
    lp.prop_cache_clear()
    g = Grid.square(256, 256 * 4e-6)
    rng = np.random.default_rng(5)
    u = torch.from_numpy(workloads.random_field(rng, (1, 256, 256)).astype(np.complex64)).cuda()
    table = 512 * 257 * 8                       # one half spectrum at M = 512
    lp.prop_cache_set_limit(6 * table)
    try:
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            y0 = host(lp.rs_propagate(u, g, 633e-9, 20e-3))
            for k in range(24):
                lp.rs_propagate(u, g, 633e-9, 21e-3 + 1e-4 * k)
                assert lp.prop_cache_info()["table_bytes"] <= 6 * table + 4 * 8 * 1024
            info = lp.prop_cache_info()
            assert info["evictions"] >= 18 and info["eviction_syncs"] >= 1
            assert info["eviction_syncs"] < info["evictions"]
            y1 = host(lp.rs_propagate(u, g, 633e-9, 20e-3))
        assert np.array_equal(y0, y1)
    finally:
        lp.prop_cache_set_limit(0)
        lp.prop_cache_clear()


def test_tables_made_on_one_stream_used_on_another(lp):
    """A spectrum generated on stream A (no host synchronisation) is used at
    once by a call on stream B: B waits for A's event on the device."""
    import torch
    lp.prop_cache_clear()
    g = Grid.square(512, 512 * 4e-6)
    rng = np.random.default_rng(6)
    u = torch.from_numpy(workloads.random_field(rng, (2, 512, 512)).astype(np.complex64)).cuda()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        with torch.cuda.stream(a):
            ya = lp.rs_propagate(u, g, 600e-9, 40e-3)
        with torch.cuda.stream(b):
            yb = lp.rs_propagate(u, g, 600e-9, 40e-3)
        torch.cuda.synchronize()
        ref = oracle.rs_propagate(u.cpu().numpy().astype(np.complex128), g, 600e-9, 40e-3)
    assert rel_l2(host(ya), ref) < 1e-6
    assert np.array_equal(host(ya), host(yb))


def test_lattice_distance_adam_memory_bounded(lp):
    """30 Adam steps on the 48 distances (and phases) of a 3 x 3 lattice at
    256^2: every step needs new kernel spectra and their z-derivatives, yet
    with a 96 MiB budget the cache stays within it and free device memory
    stays within a fixed margin from step 5 on."""
    import torch
    from paper_2310_08408_amd.lattice import Lattice, n_links
    lp.prop_cache_clear()
    limit = 96 << 20
    lp.prop_cache_set_limit(limit)
    try:
        R = C = 3
        n = 256
        g = Grid.square(n, n * 4.8e-6)
        win = Grid.square(32, 32 * 20e-9)
        lat = Lattice(R, C, g, win, 0.9, 2e-3, [True] * n_links(R, C), comps="total", eps=0.5)
        ex = oracle.gaussian_beam(g, 0.3e-3) / math.sqrt(2)
        src = torch.from_numpy(np.stack([ex]).astype(np.complex64)).cuda()
        beams = [{"wavelength": 532e-9, "sources": [(src, src) for _ in range(6)]}]
        p = lat.random_params(1, seed=7, z_range=(20e-3, 60e-3))
        opt = lp.Adam(p.tensors(), lr=2e-4)
        free, losses = [], []
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            for step in range(30):
                opt.zero_grad()
                val, _ = lat.forward(beams, p)
                val.sum().backward()
                opt.step()
                torch.cuda.synchronize()
                losses.append(float(val.detach().sum()))
                free.append(torch.cuda.mem_get_info()[0])
                info = lp.prop_cache_info()
                assert info["table_bytes"] <= limit, info
        drop = max(free[4:]) - min(free[4:])
        say(f"lattice distance Adam: loss {losses[0]:.4e} -> {losses[-1]:.4e}; cache {info}; "
            f"free-memory spread steps 5..30: {drop / 2**20:.1f} MiB")
        assert info["evictions"] > 0
        assert drop <= limit, drop
        assert all(np.isfinite(losses))
    finally:
        lp.prop_cache_set_limit(0)
        lp.prop_cache_clear()


def test_plan_fault_injection_nomem(lp):
    """PROP_PLAN_FAULT_NOMEM: plan creation fails with PROP_ENOMEM as on an
    exhausted device, frees what it allocated, pins nothing and launches
    nothing on the caller's buffers."""
    import torch
    lp.prop_cache_clear()
    g = Grid.square(64, 64 * 8e-6)
    u = torch.ones((1, 64, 64), dtype=torch.complex64, device="cuda")
    y = torch.full((1, 64, 64), 7 + 3j, dtype=torch.complex64, device="cuda")
    gi = torch.full((1, 64, 64), -1 - 1j, dtype=torch.complex64, device="cuda")
    s = lp.Setup(lp.PROP_OP_RS, g, [u], [y], [y], 600e-9, 30e-3, grad_inputs=[gi])
    before = torch.cuda.mem_get_info()[0]
    with pytest.raises(lp.PropError) as e:
        lp.Plan([s], graph=True, flags=lp.PROP_PLAN_FAULT_NOMEM)
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((y == (7 + 3j)).all()) and bool((gi == (-1 - 1j)).all())
    assert lp.prop_cache_info()["pinned"] == 0
    assert torch.cuda.mem_get_info()[0] >= before - (64 << 20)
    # the same setup without the flag works
    p = lp.Plan([s], graph=True)
    p.forward(); p.adjoint()
    torch.cuda.synchronize()
    assert not bool((y == (7 + 3j)).all())
    p.close()
