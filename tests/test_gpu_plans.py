"""Batched uneven setups through the plan API (one graph launch per
direction, or per forward+adjoint step): every setup's results equal the
single calls and the FP64 oracle (paper: Results, batches of candidate
setups evaluated per step)."""
import math
import warnings
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


def _lens(g, wl, f, sign):
    """exp(sign * i k r^2 / 2f) on grid g (thin lens, C2), FP64."""
    x, y = oracle.coords(g)
    return np.exp(sign * 1j * (2 * math.pi / wl) * (x[None, :] ** 2 + y[:, None] ** 2) / (2 * f))


def _oracle_setup(w, v_ref, gy):
    """FP64 oracle of one uneven setup: SLM phase -> RS(z) -> lens f -> CZT at
    z = f onto the window; then the adjoint chain from the window seed gy."""
    g, wl, win = w["grid"], w["wavelength"], w["window"]
    phi = np.asarray(w["phase"], np.float32).astype(np.float64)
    u = oracle.modulate(v_ref, phi)
    a = oracle.rs_propagate(u, g, wl, w["z"])
    y = oracle.czt_propagate(a * _lens(g, wl, w["f"], -1), g, win, wl, w["f"])
    ga = oracle.czt_adjoint(gy, g, win, wl, w["f"]) * _lens(g, wl, w["f"], +1)
    gu = oracle.rs_adjoint(ga, g, wl, w["z"])
    return a, y, ga, oracle.phase_grad(gu, u), gu * np.exp(-1j * phi)


def _build_plans(lp, torch, setups, win_of, graph, seed=0):
    ta, tb, keep = [], [], []
    rng = np.random.default_rng(seed)
    for w in setups:
        g = w["grid"]
        win = win_of(w)
        w["window"] = win
        v = lp.prop_source_gaussian(g, w["w0"], w["wavelength"])
        phi = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda")
        a = torch.empty_like(v)
        y = torch.empty((1, win.ny, win.nx), dtype=torch.complex64, device="cuda")
        gy_host = workloads.random_field(rng, (win.ny, win.nx)).astype(np.complex64)
        gy = torch.from_numpy(gy_host[None]).cuda()
        ga, gv = torch.empty_like(v), torch.empty_like(v)
        gphi = torch.empty_like(phi)
        ta.append(lp.Setup(lp.PROP_OP_RS, g, [v], [a], [ga], w["wavelength"], w["z"], phase=phi, grad_inputs=[gv],
                           grad_phase=gphi))
        tb.append(lp.Setup(lp.PROP_OP_CZT, g, [a], [y], [gy], w["wavelength"], w["f"], window=win, lens_f=w["f"],
                           grad_inputs=[ga]))
        keep.append(dict(w=w, v=v, phi=phi, a=a, y=y, gy=gy, gy_host=gy_host, ga=ga, gv=gv, gphi=gphi))
    return lp.Plan(ta, graph=graph), lp.Plan(tb, graph=graph), keep


def _build_chain(lp, torch, keep, graph):
    """One plan of chained setups (SLM -> RS(z) -> lens f -> CZT at z = f)
    over the tensors of `keep` (its own outputs)."""
    setups, outs = [], []
    for k in keep:
        w = k["w"]
        y, gv, gphi = torch.empty_like(k["y"]), torch.empty_like(k["v"]), torch.empty_like(k["phi"])
        setups.append(lp.Setup(lp.PROP_OP_RS_CZT, w["grid"], [k["v"]], [y], [k["gy"]], w["wavelength"], w["z"],
                               window=w["window"], lens_f=w["f"], phase=k["phi"], grad_inputs=[gv],
                               grad_phase=gphi, z2=w["f"]))
        outs.append(dict(y=y, gv=gv, gphi=gphi))
    return lp.Plan(setups, graph=graph), outs


def _check_setup(lp, k, tol_single=1e-6):
    """Plan results of one setup against single library calls and the oracle."""
    w = k["w"]
    g, wl = w["grid"], w["wavelength"]
    h = lambda t: t.cpu().numpy()[0]
    u = lp.prop_modulate(k["v"], k["phi"])
    assert rel_l2(h(k["a"]), h(lp.rs_propagate(u, g, wl, w["z"]))) < tol_single
    ref = _oracle_setup(w, oracle.gaussian_beam(g, w["w0"]), k["gy_host"].astype(np.complex128))
    errs = [rel_l2(h(k[name]), r) for name, r in zip(("a", "y", "ga", "gphi", "gv"), ref)]
    assert max(errs[:3] + errs[4:]) < 1e-5, errs
    assert errs[3] < 1e-3, errs
    return errs


@pytest.mark.parametrize("graph", [False, True])
def test_uneven_rs_lens_czt_plans(lp, graph):
    """Uneven setups: SLM phase -> RS(z) [plan A], thin lens f -> CZT at z = f
    onto a small window [plan B]; forward then adjoint, graph or eager."""
    import torch
    import warnings
    setups = _uneven(3, 6, (48, 64, 96, 130))
    for w in setups:
        w["w0"] = 0.6e-3
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        pa, pb, keep = _build_plans(lp, torch, setups, lambda w: Grid.square(40, 40 * 0.5e-6), graph)
        pc, chain = _build_chain(lp, torch, keep, graph)
        for rep in range(2):  # replays must agree
            pa.forward(); pb.forward(); pb.adjoint(); pa.adjoint()
            pc.forward(); pc.adjoint()
            torch.cuda.synchronize()
            worst = np.max([_check_setup(lp, k) for k in keep], axis=0)
            say(f"graph={graph} replay {rep}: {len(keep)} setups agree with single calls and the oracle; "
                f"worst rel-L2 a/y/ga/gphi/gv = " + " ".join(f"{e:.1e}" for e in worst))
            # the chained setups run the same kernels in the same order
            for k, c in zip(keep, chain):
                for name in ("y", "gv", "gphi"):
                    assert torch.equal(k[name], c[name]), (name, k["w"]["index"])
    pa.close(); pb.close(); pc.close()


@pytest.fixture(scope="module")
def uneven96(lp):
    """The 96-setup uneven workload (N in {512..2048}, 1024^2 window) as one
    plan of chained setups -- SLM -> RS(z) -> lens f -> CZT at z = f -- with
    forward and adjoint as one graph launch (prop_plan_step); timed over
    replays, then every setup's results copied to the host."""
    import time
    import torch
    setups = _uneven(0, 96, workloads.UNEVEN_SIZES)
    say("uneven 96: sizes", {n: sum(1 for w in setups if w["grid"].nx == n) for n in workloads.UNEVEN_SIZES})
    rng = np.random.default_rng(0)
    keep, chain = [], []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        t0 = time.perf_counter()
        for w in setups:
            g, win = w["grid"], w["window"]
            v = lp.prop_source_gaussian(g, w["w0"], w["wavelength"])
            phi = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda")
            gy_host = workloads.random_field(rng, (win.ny, win.nx)).astype(np.complex64)
            keep.append(dict(w=w, v=v, phi=phi, gy=torch.from_numpy(gy_host[None]).cuda(), gy_host=gy_host,
                             y=torch.empty((1, win.ny, win.nx), dtype=torch.complex64, device="cuda")))
        plan, chain = _build_chain(lp, torch, keep, graph=True)
        torch.cuda.synchronize()
        say(f"  chained plan built (spectra, chirps) in {time.perf_counter() - t0:.2f} s")
        for _ in range(2):
            plan.step()
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        say(f"  96 setups forward+adjoint: {ms:.2f} ms per step, one graph launch "
            f"({96e3 / ms:.1f} setup-gradients/s)")
    h = lambda t: t.cpu().numpy()[0]
    res = [dict(w=k["w"], gy_host=k["gy_host"], y=h(c["y"]), gv=h(c["gv"]), gphi=h(c["gphi"])) for k, c in
           zip(keep, chain)]
    plan.close()
    return res


def _oracle_chain(w, gy):
    """FP64 oracle of one chained setup: y = CZT_f(L RS_z(V e^{i phi})) and
    the gradients of <gy, y> with respect to V (g_v) and phi."""
    g, wl, win = w["grid"], w["wavelength"], w["window"]
    phi = np.asarray(w["phase"], np.float32).astype(np.float64)
    v = oracle.gaussian_beam(g, w["w0"])
    u = oracle.modulate(v, phi)
    y = oracle.czt_propagate(oracle.rs_propagate(u, g, wl, w["z"]) * _lens(g, wl, w["f"], -1), g, win, wl, w["f"])
    gu = oracle.rs_adjoint(oracle.czt_adjoint(gy, g, win, wl, w["f"]) * _lens(g, wl, w["f"], +1), g, wl, w["z"])
    return y, gu * np.exp(-1j * phi), oracle.phase_grad(gu, u)


@pytest.mark.parametrize("graph", [False, True])
def test_plan_step_equals_forward_then_adjoint(lp, graph):
    """prop_plan_step (forward then adjoint; one graph launch for a graph
    plan) gives the results of prop_plan_forward followed by
    prop_plan_adjoint bit for bit, over three replays, on chained setups of
    uneven sizes."""
    import torch
    setups = _uneven(5, 6, (48, 64, 96, 130))
    rng = np.random.default_rng(5)
    keep = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for w in setups:
            w["w0"] = 0.6e-3
            w["window"] = win = Grid.square(40, 40 * 0.5e-6)
            v = lp.prop_source_gaussian(w["grid"], w["w0"], w["wavelength"])
            phi = torch.tensor(w["phase"][None], dtype=torch.float32, device="cuda")
            gy = torch.from_numpy(workloads.random_field(rng, (1, win.ny, win.nx)).astype(np.complex64)).cuda()
            keep.append(dict(w=w, v=v, phi=phi, gy=gy, y=torch.empty_like(gy)))
        p1, o1 = _build_chain(lp, torch, keep, graph)
        p2, o2 = _build_chain(lp, torch, keep, graph)
        for rep in range(3):
            p1.forward(); p1.adjoint()
            p2.step()
            torch.cuda.synchronize()
            for a, b in zip(o1, o2):
                for name in ("y", "gv", "gphi"):
                    assert torch.equal(a[name], b[name]), (rep, name)
    say(f"graph={graph}: plan step = forward + adjoint bit for bit over {len(keep)} setups, 3 replays")
    p1.close(); p2.close()


@pytest.mark.parametrize("part", range(4))
def test_uneven_96_chained_plan_vs_oracle(uneven96, part):
    """Every one of the 96 setups of the chained plan (a quarter per test)
    against the FP64 oracle: field on the window, input gradient and SLM
    phase gradient."""
    import os
    import scipy.fft
    worst = np.zeros(3)
    with scipy.fft.set_workers(min(16, os.cpu_count() or 1)):
        for r in uneven96[part * 24:(part + 1) * 24]:
            ref = _oracle_chain(r["w"], r["gy_host"].astype(np.complex128))
            errs = np.array([rel_l2(r[name], x) for name, x in zip(("y", "gv", "gphi"), ref)])
            worst = np.maximum(worst, errs)
            assert errs[0] < 1e-5 and errs[1] < 1e-5 and errs[2] < 1e-3, (r["w"]["index"], r["w"]["grid"].nx, errs)
    say(f"uneven 96 setups {24 * part}..{24 * part + 23} vs oracle: worst rel-L2 y/g_v/g_phi = "
        + " ".join(f"{e:.1e}" for e in worst))


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


def _tune_plans(lp, torch, autotune, graph, seed=11):
    g = Grid.square(512, 4e-3)
    win = Grid.square(512, 40e-6)
    rng = np.random.default_rng(seed)
    v = torch.from_numpy(workloads.random_field(rng, (2, 512, 512)).astype(np.complex64)).cuda()
    y_rs, y_czt = torch.empty_like(v), torch.empty_like(v)
    g_rs, g_czt = torch.empty_like(v), torch.empty_like(v)
    s1 = lp.Setup(lp.PROP_OP_RS, g, [v], [y_rs], [y_rs], 600e-9, 30e-3, grad_inputs=[g_rs])
    s2 = lp.Setup(lp.PROP_OP_CZT, g, [v], [y_czt], [y_czt], 600e-9, 40e-3, window=win, grad_inputs=[g_czt])
    return lp.Plan([s1, s2], graph=graph, autotune=autotune), (v, y_rs, y_czt, g_rs, g_czt), (g, win)


@pytest.mark.parametrize("graph", [False, True])
def test_autotuned_plan(lp, graph, tmp_path):
    """PROP_PLAN_AUTOTUNE times the lines-per-workgroup variants and the
    alternative radix schedules of the column and Bluestein passes at the
    first execution and records each choice (here in a fresh tuning cache
    file).  Every replay of the tuned plan is bit-identical to its first
    execution; against the untuned plan and the FP64 oracle the results
    agree to FP32 rounding (a different schedule rounds differently)."""
    import torch
    lp.prop_cache_clear()
    cache = tmp_path / "tune.txt"
    assert lp.prop_tune_cache_path(str(cache)) == 0
    p0, t0, (g, win) = _tune_plans(lp, torch, False, graph)
    p1, t1, _ = _tune_plans(lp, torch, True, graph)
    assert torch.equal(t0[0], t1[0])
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        first = None
        for rep in range(3):
            p0.forward(); p0.adjoint(); p1.forward(); p1.adjoint()
            torch.cuda.synchronize()
            got = [t.cpu().numpy() for t in t1[1:]]
            if first is None:
                first = got
            for a, b in zip(first, got):
                assert np.array_equal(a, b), f"replay {rep}"
            for a, b in zip(t0[1:], t1[1:]):
                assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) < 1e-5
    report = lp.prop_autotune_report()
    say(report)
    for kind in ("rs_cols n=1024", "czt_cols n=1024", "czt_rows n=1024"):
        assert kind in report
    assert "timed" in report and "from file" not in report
    recs = [l for l in cache.read_text().splitlines() if l.startswith("libprop-tune 1 ")]
    assert len(recs) >= 3, recs   # RS columns, Bluestein rows and columns (shared by both directions)
    v = t0[0].cpu().numpy().astype(np.complex128)
    ref_rs = oracle.rs_propagate(v, g, 600e-9, 30e-3)
    assert rel_l2(t1[1].cpu().numpy(), ref_rs) < 1e-5
    p0.close(); p1.close()
    lp.prop_tune_cache_path(None)


def _rs_plan(lp, torch, n, seed):
    g = Grid.square(n, 4e-3)
    rng = np.random.default_rng(seed)
    v = torch.from_numpy(workloads.random_field(rng, (1, n, n)).astype(np.complex64)).cuda()
    y, gi = torch.empty_like(v), torch.empty_like(v)
    s = lp.Setup(lp.PROP_OP_RS, g, [v], [y], [y], 600e-9, 30e-3, grad_inputs=[gi])
    return lp.Plan([s], graph=False, autotune=True), (v, y, gi), g


@pytest.mark.parametrize("n", [512, 1024, 2048])
def test_rs_column_variants_pinned_from_file(lp, tmp_path, n):
    """Every candidate of the RS column pass at one shape, pinned in turn
    through a tuning cache record (the persistent pass for these
    exact-half FP32 lengths): the lines-per-workgroup variants of the
    built-in schedule (0-2) give the same bits as variant 0 in the forward
    and the adjoint, the alternative schedule's (3-5) agree to FP32
    rounding, and variant 0 matches the oracle."""
    import torch
    lp.prop_cache_clear()
    probe = tmp_path / "probe.txt"
    lp.prop_tune_cache_path(str(probe))
    p, t, g = _rs_plan(lp, torch, n, 5)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        p.forward()
    torch.cuda.synchronize()
    p.close()
    recs = [l.split() for l in probe.read_text().splitlines() if l.startswith("libprop-tune")]
    rs = [r for r in recs if r[4] == "0" and r[5] == str(2 * n)]
    assert rs, recs
    outs = {}
    for var in range(6):
        f = tmp_path / f"v{var}.txt"
        f.write_text(" ".join(rs[0][:10] + [str(var)]) + "\n")
        lp.prop_cache_clear()
        if lp.prop_tune_cache_path(str(f)) != 1:
            continue  # not a candidate of this shape
        p, t, g = _rs_plan(lp, torch, n, 5)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            p.forward(); p.adjoint()
        torch.cuda.synchronize()
        line = [l for l in lp.prop_autotune_report().splitlines() if f"rs_cols n={2 * n}" in l][0]
        assert f"variant {var}" in line and "from file" in line, line
        outs[var] = (t[1].cpu().numpy(), t[2].cpu().numpy())
        p.close()
    say(f"RS columns n={2 * n}: variants pinned {sorted(outs)}")
    assert 0 in outs, sorted(outs)
    for var, (y, gi) in outs.items():
        if var < 3:
            assert np.array_equal(y, outs[0][0]) and np.array_equal(gi, outs[0][1]), var
        else:
            assert rel_l2(y, outs[0][0]) < 1e-5 and rel_l2(gi, outs[0][1]) < 1e-5, var
    if n <= 1024:
        v0 = t[0].cpu().numpy().astype(np.complex128)
        assert rel_l2(outs[0][0], oracle.rs_propagate(v0, g, 600e-9, 30e-3)) < 1e-5
    lp.prop_tune_cache_path(None)
    lp.prop_cache_clear()


def test_tuning_cache_file_is_read_and_corruption_ignored(lp, tmp_path):
    """A record in the tuning cache file fixes a shape's choice (here the
    alternative 8x16x8 schedule of the 1024-point RS column pass) without
    timing; malformed lines, unknown versions, variants that are not
    candidates of their shape and other architectures are skipped, and those
    shapes are timed anew.  Results stay within FP32 rounding of the
    oracle."""
    import torch
    lp.prop_cache_clear()
    # the shapes of the plan: learn them (and the architecture) from a tuning run
    probe = tmp_path / "probe.txt"
    lp.prop_tune_cache_path(str(probe))
    p, t, (g, win) = _tune_plans(lp, torch, True, False, seed=3)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        p.forward(); p.adjoint()
    torch.cuda.synchronize()
    p.close()
    recs = [l.split() for l in probe.read_text().splitlines() if l.startswith("libprop-tune")]
    rs = [r for r in recs if r[4] == "0" and r[5] == "1024"]
    assert rs, recs
    arch = rs[0][2]
    forced = rs[0][:10] + ["3"]                          # RS columns at 1024 on the alternative schedule
    bad_variant = rs[0][:10] + ["5"]                     # lines variant 2 of a 1024-point alt: valid only if it exists
    good = tmp_path / "good.txt"
    good.write_text("# tuning cache\n" + " ".join(forced) + "\n")
    lp.prop_cache_clear()
    assert lp.prop_tune_cache_path(str(good)) == 1 and lp.prop_tune_cache_rejected() == 0
    p, t, _ = _tune_plans(lp, torch, True, False, seed=3)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        p.forward(); p.adjoint()
    torch.cuda.synchronize()
    report = lp.prop_autotune_report()
    say(report)
    line = [l for l in report.splitlines() if "rs_cols n=1024" in l][0]
    assert "variant 3" in line and "8x16x8" in line and "from file" in line
    v = t[0].cpu().numpy().astype(np.complex128)
    assert rel_l2(t[1].cpu().numpy(), oracle.rs_propagate(v, g, 600e-9, 30e-3)) < 1e-5
    p.close()
    corrupt = tmp_path / "corrupt.txt"
    corrupt.write_text("\n".join([
        "libprop-tune 1",                                               # truncated
        "libprop-tune 2 " + " ".join(forced[2:]),                       # unknown version
        " ".join(rs[0][:10] + ["9"]),                                   # variant out of range
        " ".join(rs[0][:5] + ["4096"] + rs[0][6:10] + ["3"]),           # 4096 has no alternative schedule
        "\x00\x01 garbage \xff",
        " ".join(["libprop-tune", "1", "gfx000"] + forced[3:]),         # another architecture: not used here
    ]) + "\n", errors="surrogateescape")
    lp.prop_cache_clear()
    n_ok = lp.prop_tune_cache_path(str(corrupt))
    assert n_ok == 1 and lp.prop_tune_cache_rejected() == 5, (n_ok, lp.prop_tune_cache_rejected())
    p, t, _ = _tune_plans(lp, torch, True, False, seed=3)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        p.forward(); p.adjoint()
    torch.cuda.synchronize()
    report = lp.prop_autotune_report()
    assert "from file" not in report and "timed" in report
    assert rel_l2(t[1].cpu().numpy(), oracle.rs_propagate(v, g, 600e-9, 30e-3)) < 1e-5
    p.close()
    del bad_variant, arch
    lp.prop_tune_cache_path(None)
    lp.prop_cache_clear()
