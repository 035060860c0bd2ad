"""The Python binding checks every tensor argument (device, contiguity,
dtype, [batch, ny, nx] shape) before a pointer reaches the C ABI: a
mismatched argument raises ValueError and nothing is launched."""
import numpy as np
import pytest

from workloads import Grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2310_08408_amd as lp
    lp.library()
    return lp


def _c(*shape, dt=None):
    import torch
    return torch.zeros(shape, dtype=dt or torch.complex64, device="cuda")


def test_mismatched_arguments_raise_before_launch(lp):
    import torch
    g = Grid(32, 24, 4e-6, 4e-6)
    win = Grid(16, 16, 0.5e-6, 0.5e-6)
    u = _c(2, 24, 32)
    sentinel = torch.full((2, 24, 32), 5.0, dtype=torch.float32, device="cuda")
    cases = [
        # adjoint seed with one plane fewer than the field
        lambda: lp.rs_adjoint_phase_grad(_c(1, 24, 32), u, g, 6e-7, 3e-2, grad=sentinel),
        # CZT seed on the input grid instead of the window
        lambda: lp.czt_adjoint_phase_grad(_c(2, 24, 32), u, g, win, 6e-7, 3e-2, grad=sentinel),
        # phase gradient of the wrong precision or length
        lambda: lp.rs_adjoint_phase_grad(u.clone(), u, g, 6e-7, 3e-2, grad=sentinel.double()),
        lambda: lp.rs_adjoint_phase_grad(u.clone(), u, g, 6e-7, 3e-2, grad=sentinel[:1]),
        lambda: lp.rs_adjoint_phase_grad(u.clone(), u, g, 6e-7, 3e-2, grad=sentinel, g_u=_c(2, 24, 31)),
        # vector components of mixed precision or shape
        lambda: lp.vrs_propagate(u, _c(2, 24, 32, dt=torch.complex128), g, 6e-7, 3e-2),
        lambda: lp.vrs_adjoint(u, u, _c(1, 24, 32), g, 6e-7, 3e-2),
        lambda: lp.vczt_propagate(u, _c(2, 24, 31), g, win, 6e-7, 3e-2),
        lambda: lp.vczt_adjoint(_c(2, 16, 16), _c(2, 16, 16), _c(2, 24, 32), g, win, 6e-7, 3e-2),
        # distance gradients with seeds on the wrong grid
        lambda: lp.rs_grad_z(u, _c(2, 16, 16), g, 6e-7, 3e-2),
        lambda: lp.czt_grad_z(u, _c(2, 16, 16), g, win, 6e-7, 3e-2, u_out=_c(2, 24, 32)),
        # element calls: host tensors, wrong out, wrong phase length
        lambda: lp.prop_modulate(u, torch.zeros((2, 24, 32), dtype=torch.float32), out=None),
        lambda: lp.prop_modulate(u, sentinel, out=_c(1, 24, 32)),
        lambda: lp.prop_modulate(u, torch.zeros((3, 24, 32), dtype=torch.float32, device="cuda")),
        lambda: lp.prop_phase_grad(_c(2, 24, 16), u),
        lambda: lp.prop_phase_grad_sum(u, u, grad=sentinel),
        lambda: lp.prop_waveplate_batched_adjoint(u.cpu(), u, u, u, torch.zeros((2, 2), dtype=torch.float64,
                                                                               device="cuda")),
        lambda: lp.prop_waveplate_batched(u, u, torch.zeros((2, 2), dtype=torch.float64)),
        lambda: lp.prop_beam_splitter_adjoint([u], [u.cpu()], [u], None,
                                              torch.zeros(2, dtype=torch.float64, device="cuda")),
        lambda: lp.prop_beam_splitter([u], [_c(2, 24, 32, dt=torch.complex128)], torch.zeros(2, dtype=torch.float64,
                                                                                        device="cuda")),
        # out= planes of the element calls with the wrong shape, precision or count
        lambda: lp.prop_waveplate_batched(u, u, torch.zeros((2, 2), dtype=torch.float64, device="cuda"),
                                          out=(_c(2, 24, 32), _c(1, 24, 32))),
        lambda: lp.prop_waveplate_batched_adjoint(u, u, u, u, torch.zeros((2, 2), dtype=torch.float64, device="cuda"),
                                                  out=(_c(2, 24, 32, dt=torch.complex128), _c(2, 24, 32))),
        lambda: lp.prop_beam_splitter([u, u], [u, u], torch.zeros(2, dtype=torch.float64, device="cuda"),
                                      out=([_c(2, 24, 32), _c(2, 24, 32)], [_c(2, 24, 32)])),
        lambda: lp.prop_beam_splitter_adjoint([u, u], [u, u], [u, u], None,
                                              torch.zeros(2, dtype=torch.float64, device="cuda"), (True, False),
                                              out=([_c(2, 24, 32), _c(2, 24, 31)], None)),
        lambda: lp.prop_spot_loss(_c(2, 16, 16), _c(2, 16, 16), _c(1, 16, 16), win, 6e-7),
        lambda: lp.prop_density_loss([_c(2, 16, 16), _c(2, 16, 15)], 0.5),
        lambda: lp.prop_scale_items([u, _c(1, 24, 32)], torch.ones(2, dtype=torch.float64, device="cuda")),
        lambda: lp.rs_propagate(u, g, 6e-7, 3e-2, out=_c(2, 24, 32, dt=torch.complex128)),
        lambda: lp.czt_propagate(u[:, :, ::2], g, win, 6e-7, 3e-2),
    ]
    for k, case in enumerate(cases):
        with pytest.raises((ValueError, TypeError)):
            case()
    torch.cuda.synchronize()
    assert bool((sentinel == 5.0).all()), "a rejected call wrote its output"


def test_plan_rejects_mismatched_setups(lp):
    import torch
    g = Grid(32, 32, 4e-6, 4e-6)
    win = Grid(16, 16, 0.5e-6, 0.5e-6)
    v64 = _c(1, 32, 32)
    v128 = _c(1, 32, 32, dt=torch.complex128)
    ok = lp.Setup(lp.PROP_OP_RS, g, [v128], [v128.clone()], [v128.clone()], 6e-7, 3e-2)
    bad = [
        # complex64 setup inside a complex128 plan
        ([lp.Setup(lp.PROP_OP_RS, g, [v64], [v64.clone()], [v64.clone()], 6e-7, 3e-2)], torch.complex128),
        # CZT output on the input grid instead of the window
        ([lp.Setup(lp.PROP_OP_CZT, g, [v64], [v64.clone()], [v64.clone()], 6e-7, 3e-2, window=win)],
         torch.complex64),
        # CZT without a window
        ([lp.Setup(lp.PROP_OP_CZT, g, [v64], [_c(1, 16, 16)], [_c(1, 16, 16)], 6e-7, 3e-2)], torch.complex64),
        # phase of the wrong precision, gradient of the wrong batch
        ([lp.Setup(lp.PROP_OP_RS, g, [v64], [v64.clone()], [v64.clone()], 6e-7, 3e-2,
                   phase=torch.zeros((1, 32, 32), dtype=torch.float64, device="cuda"))], torch.complex64),
        ([lp.Setup(lp.PROP_OP_RS, g, [v64], [v64.clone()], [v64.clone()], 6e-7, 3e-2,
                   grad_inputs=[_c(2, 32, 32)])], torch.complex64),
        # vector op with one input
        ([lp.Setup(lp.PROP_OP_VRS, g, [v64], [v64.clone()] * 3, [v64.clone()] * 3, 6e-7, 3e-2)], torch.complex64),
        # a host tensor among the outputs
        ([lp.Setup(lp.PROP_OP_RS, g, [v64], [v64.cpu()], [v64.clone()], 6e-7, 3e-2)], torch.complex64),
        # mixed setups
        ([ok, lp.Setup(lp.PROP_OP_RS, g, [v64], [v64.clone()], [v64.clone()], 6e-7, 3e-2)], torch.complex128),
    ]
    for setups, dt in bad:
        with pytest.raises((ValueError, TypeError)):
            lp.Plan(setups, dtype=dt)
    p = lp.Plan([ok], dtype=torch.complex128)
    p.close()


def test_sum_items(lp):
    """prop_sum_items: the per-item sum of a batch-shared parameter's
    gradients, in item order in FP64 on the device."""
    import torch
    rng = np.random.default_rng(4)
    x = rng.standard_normal((7, 5, 2))
    got = lp.prop_sum_items(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = np.zeros((5, 2))
    for i in range(7):
        ref = ref + x[i]
    assert np.array_equal(got, ref)
    assert float(lp.prop_sum_items(torch.tensor([1.5, -2.0, 4.0], dtype=torch.float64, device="cuda"))) == 3.5
    with pytest.raises(ValueError):
        lp.prop_sum_items(torch.zeros(3, dtype=torch.float32, device="cuda"))
