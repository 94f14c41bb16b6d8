"""The hand-written backward behind torch.autograd.Function, on the GPU.

Checked three ways on the 256x256, S=32, 12-blade workload and a dynamic case:
against the oracle's gradient, against central finite differences of the loss the
forward kernels compute (the data term is quadratic, so the central difference is
exact up to rounding), and by the dot-product adjoint identity through autograd.
"""

import numpy as np
import pytest

import oracle as O
from parity import assert_close
from synth import configs

pytestmark = pytest.mark.gpu


def _t(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def data_loss(vol, plan, y):
    """The test's loss: 0.5 * sum |M (A vol) - M y|^2 over the residual the library returns
    (float64 accumulation in torch; the objective itself is the test's, not the library's)."""
    import torch

    from paper_2311_13177_amd import autograd as AG

    r = AG.lifted_forward(vol, plan, y)
    return 0.5 * torch.sum(torch.view_as_real(r).to(torch.float64) ** 2)


def _rand(rng, shape, scale=1.0):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale).astype(np.complex64)


@pytest.mark.parametrize("name", ["static_256", "dynamic_40"])
def test_autograd_gradient_fd_and_oracle(gpu_lib, name):
    import torch

    from paper_2311_13177_amd import autograd as AG
    from paper_2311_13177_amd import binding as B

    if name == "static_256":
        case = configs.static_256()
    else:
        case = configs.small_case(n=40, n_spec=5, n_time=3, n_blades=6, lines=8)
    plan = B.Plan.from_geometry(case.geometry())
    geom = O.Geometry.from_dict(case.geometry())
    rng = np.random.default_rng(21)
    y = O.simulate_measurements(case)
    v0 = _rand(rng, plan.volume_shape, 0.05)
    vol = _t(v0).requires_grad_(True)
    yt = _t(y)
    loss = data_loss(vol, plan, yt)
    loss.backward()
    g = vol.grad.cpu().numpy().astype(np.complex128)
    g_or, ld_or = O.gradient(v0.astype(np.complex128), geom, y, 0.0, 1e-3)
    assert_close(g, g_or, 1e-4)
    assert abs(loss.item() - ld_or) <= 1e-4 * ld_or
    # central finite difference along random directions
    with torch.no_grad():
        for k in range(2):
            h = _rand(rng, plan.volume_shape, 0.05)
            ht = _t(h)
            lp = data_loss(vol + ht, plan, yt).item()
            lm = data_loss(vol - ht, plan, yt).item()
            fd = (lp - lm) / 2.0
            an = float(np.real(np.vdot(g, h.astype(np.complex128))))
            assert abs(fd - an) <= 1e-3 * max(abs(an), 1e-12) + 1e-6 * abs(lp), (fd, an)


def test_autograd_dot_product_identity(gpu_lib):
    import torch

    from paper_2311_13177_amd import autograd as AG
    from paper_2311_13177_amd import binding as B

    case = configs.static_256()
    plan = B.Plan.from_geometry(case.geometry())
    rng = np.random.default_rng(22)
    x = _t(_rand(rng, plan.volume_shape)).requires_grad_(True)
    k = _t(_rand(rng, plan.blade_shape) * plan.masks())
    ax = AG.lifted_forward(x, plan)
    (ahk,) = torch.autograd.grad(ax, x, grad_outputs=k)
    lhs = np.vdot(k.cpu().numpy().astype(np.complex128), ax.detach().cpu().numpy().astype(np.complex128))
    rhs = np.vdot(ahk.cpu().numpy().astype(np.complex128), x.detach().cpu().numpy().astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_regulariser_function_matches_oracle(gpu_lib):
    from paper_2311_13177_amd import autograd as AG
    from paper_2311_13177_amd import binding as B

    case = configs.small_case(n=48, n_spec=6, n_blades=4, lines=12)
    plan = B.Plan.from_geometry(case.geometry())
    geom = O.Geometry.from_dict(case.geometry())
    rng = np.random.default_rng(23)
    y = O.simulate_measurements(case)
    v0 = _rand(rng, plan.volume_shape, 0.05)
    vol = _t(v0).requires_grad_(True)
    loss = data_loss(AG.Regulariser.apply(vol, plan, 1e-2, 1e-3, 1e-3), plan, _t(y))
    loss.backward()
    g_or, _ = O.gradient(v0.astype(np.complex128), geom, y, 1e-2, 1e-3, 1e-3)
    g = vol.grad.cpu().numpy().astype(np.complex128)
    assert_close(g, g_or, 1e-4)


def test_blade_aligned_autograd_matches_oracle_and_fd(gpu_lib):
    # loss = 0.5 sum |A_nu vol - y|^2 through BladeAlignedForward: its gradient against the
    # oracle's gridding gradient, and a central difference of the loss along a random
    # direction (exact for a quadratic up to rounding)
    import torch

    from oracle import nonuniform as N
    from paper_2311_13177_amd import autograd as AG
    from paper_2311_13177_amd import binding as B

    case = configs.small_case(n=48, n_spec=4, n_time=3, n_blades=5, lines=10)
    plan = B.Plan.from_geometry(case.geometry())
    geom = O.Geometry.from_dict(case.geometry())
    rng = np.random.default_rng(31)
    vol = _rand(rng, plan.volume_shape, 0.3)
    shp = B.nu_shape(plan)
    y = _rand(rng, shp)
    x = _t(vol).requires_grad_(True)
    r = AG.blade_aligned_forward(x, plan, _t(y))
    loss = 0.5 * torch.sum(torch.view_as_real(r).to(torch.float64) ** 2)
    loss.backward()
    g = x.grad.cpu().numpy().astype(np.complex128)
    want, val = N.gradient_nu(vol.astype(np.complex128), geom, [y[b].astype(np.complex128) for b in range(shp[0])],
                              exact=False)
    assert_close(g, want, 1e-4)
    assert abs(float(loss.detach()) - val) <= 1e-4 * val
    d = _rand(rng, plan.volume_shape)
    h = 1e-2

    def f(v):
        with torch.no_grad():
            rr = B.vp_nu_forward(plan, _t(v), _t(y)).cpu().numpy().astype(np.complex128)
        return 0.5 * float(np.sum(np.abs(rr) ** 2))

    fd = (f(vol + h * d) - f(vol - h * d)) / (2 * h)
    an = float(np.sum((np.conj(g) * d.astype(np.complex128)).real))
    assert abs(fd - an) <= 1e-3 * abs(an)
