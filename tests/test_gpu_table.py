"""Checkpointed optical-table chain on the GPU (SLM -> RS -> SLM -> two wave
plates -> NA 0.9 objective -> spot size + E_z fraction) against the FP64
oracle's uncheckpointed chain, at a small size for several parameter sets and
at the full 2048^2 / batch-32 workload (paper: Results, setups discovered from
SLMs, retarders and a high-NA lens; Methods, gradients)."""
import math
import sys
import time

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


def _run_table(torch, g, win, wl, w0, z, na, f, phi1, phi2, wp1, wp2, dtype):
    from paper_2310_08408_amd.table import OpticalTable
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    t = OpticalTable(g, win, wl, w0, z, na, f, batch=phi1.shape[0], dtype=dtype, w_fz=1.0)
    p1 = torch.as_tensor(phi1, dtype=rdt).cuda()
    p2 = torch.as_tensor(phi2, dtype=rdt).cuda()
    loss = t.forward(p1, p2, wp1, wp2)
    g1, g2, d1, d2 = t.backward()
    torch.cuda.synchronize()
    return loss.cpu().numpy(), g1.cpu().numpy(), g2.cpu().numpy(), d1.cpu().numpy(), d2.cpu().numpy()


@pytest.mark.parametrize("kind", ["c64", "c128"])
def test_table_small_vs_oracle(lp, kind):
    import torch
    dt = torch.complex64 if kind == "c64" else torch.complex128
    n, b = 64, 3
    g = Grid.square(n, n * 20e-6)
    win = Grid(40, 36, 60e-9, 70e-9, 0.05e-6, 0)
    wl, z, na, w0 = 635e-9, 3e-3, 0.9, 300e-6
    f = (n * 20e-6 / 2) / na
    rng = np.random.default_rng(7)
    phi1, phi2 = (rng.uniform(-math.pi, math.pi, (b, n, n)) for _ in range(2))
    if kind == "c64":
        phi1, phi2 = (p.astype(np.float32).astype(np.float64) for p in (phi1, phi2))
    wps = [tuple(float(x) for x in rng.uniform(-math.pi, math.pi, 4)) for _ in range(b)]
    wp1 = [(w[0], w[1]) for w in wps]
    wp2 = [(w[2], w[3]) for w in wps]
    say("table small", kind)
    loss, g1, g2, d1, d2 = _run_table(torch, g, win, wl, w0, z, na, f, phi1, phi2, wp1, wp2, dt)
    v = oracle.gaussian_beam(g, w0) / math.sqrt(2.0)
    tol_f, tol_g = (1e-5, 1e-3) if kind == "c64" else (1e-11, 1e-9)
    for s in range(b):
        ref = oracle.table_chain(v, phi1[s], phi2[s], wp1[s], wp2[s], g, win, wl, z, na, f, 1.0)
        e_loss = abs(loss[s] - ref[0]) / abs(ref[0])
        e1, e2 = rel_l2(g1[s], ref[1]), rel_l2(g2[s], ref[2])
        e_wp = max(abs(d1[s][k] - ref[3][k]) / max(1.0, abs(ref[3][k])) for k in range(2))
        e_wp = max(e_wp, max(abs(d2[s][k] - ref[4][k]) / max(1.0, abs(ref[4][k])) for k in range(2)))
        say(f"  set {s}: loss {e_loss:.2e} g_phi1 {e1:.2e} g_phi2 {e2:.2e} g_wp {e_wp:.2e}")
        assert e_loss < tol_f
        assert e1 < tol_g and e2 < tol_g and e_wp < tol_g


def test_table_2048_batch32(lp):
    """The 32-set table at 2048^2: FP32 against FP64 on the GPU for every set,
    and set 0 of both against the full FP64 oracle chain."""
    import torch
    sets = list(workloads.table_32(0))
    s0 = sets[0]
    g, win, wl, w0, z, na, f = (s0[k] for k in ("grid", "window", "wavelength", "w0", "z", "na", "f"))
    phi1 = np.stack([s["phase1"] for s in sets]).astype(np.float32)
    phi2 = np.stack([s["phase2"] for s in sets]).astype(np.float32)
    wp1 = [s["wp1"] for s in sets]
    wp2 = [s["wp2"] for s in sets]
    say("table 2048 x 32 fp32 ...")
    _run_table(torch, g, win, wl, w0, z, na, f, phi1[:1], phi2[:1], wp1[:1], wp2[:1], torch.complex64)
    t0 = time.perf_counter()
    r32 = _run_table(torch, g, win, wl, w0, z, na, f, phi1, phi2, wp1, wp2, torch.complex64)
    say(f"  fp32 forward+backward, 32 sets: {time.perf_counter() - t0:.3f} s (includes host copies)")
    torch.cuda.empty_cache()
    say("table 2048 x 32 fp64 ...")
    r64 = _run_table(torch, g, win, wl, w0, z, na, f, phi1.astype(np.float64), phi2.astype(np.float64), wp1, wp2,
                     torch.complex128)
    torch.cuda.empty_cache()
    worst = [0.0] * 4
    for s in range(32):
        worst[0] = max(worst[0], abs(r32[0][s] - r64[0][s]) / abs(r64[0][s]))
        worst[1] = max(worst[1], rel_l2(r32[1][s].astype(np.float64), r64[1][s]))
        worst[2] = max(worst[2], rel_l2(r32[2][s].astype(np.float64), r64[2][s]))
        worst[3] = max(worst[3], np.abs(r32[3][s] - r64[3][s]).max() / max(1.0, np.abs(r64[3][s]).max()),
                       np.abs(r32[4][s] - r64[4][s]).max() / max(1.0, np.abs(r64[4][s]).max()))
    say(f"  fp32 vs fp64 over 32 sets: loss {worst[0]:.2e} g_phi1 {worst[1]:.2e} g_phi2 {worst[2]:.2e} "
        f"g_wp {worst[3]:.2e}")
    assert worst[0] < 1e-5 and max(worst[1:]) < 1e-3
    say("  oracle chain for set 0 ...")
    v = oracle.gaussian_beam(g, w0) / math.sqrt(2.0)
    ref = oracle.table_chain(v, phi1[0].astype(np.float64), phi2[0].astype(np.float64), wp1[0], wp2[0], g, win, wl,
                             z, na, f, 1.0)
    for name, r, tf, tg in (("fp32", r32, 1e-5, 1e-3), ("fp64", r64, 1e-10, 1e-8)):
        e = (abs(r[0][0] - ref[0]) / abs(ref[0]), rel_l2(r[1][0].astype(np.float64), ref[1]),
             rel_l2(r[2][0].astype(np.float64), ref[2]),
             max(abs(r[3][0][k] - ref[3][k]) / max(1.0, abs(ref[3][k])) for k in range(2)),
             max(abs(r[4][0][k] - ref[4][k]) / max(1.0, abs(ref[4][k])) for k in range(2)))
        say(f"  {name} set 0 vs oracle: loss {e[0]:.2e} g_phi1 {e[1]:.2e} g_phi2 {e[2]:.2e} g_wp1 {e[3]:.2e} "
            f"g_wp2 {e[4]:.2e}")
        assert e[0] < tf and max(e[1:]) < tg
