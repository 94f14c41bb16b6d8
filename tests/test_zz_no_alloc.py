"""vp_forward_noalloc: the forward model with its blade images in the library's fixed
device scratch array, against vp_forward (same kernels, so the same bits), on two calls
in a row with the second one smaller, then the error paths."""

import numpy as np
import pytest

import oracle as O
from synth import configs

pytestmark = pytest.mark.gpu


def _vol(plan, seed):
    rng = np.random.default_rng(seed)
    shape = plan.volume_shape
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def test_forward_noalloc_matches_forward(gpu_lib):
    import torch
    from paper_2311_13177_amd import binding as B

    big = configs.small_case(n=96, n_spec=6, n_time=3, n_blades=7, lines=12, f=2.5, seed=21)
    small = configs.small_case(n=48, n_spec=4, n_blades=3, lines=8, seed=22)
    for case, seed in ((big, 1), (small, 2)):
        plan = B.Plan.from_geometry(case.geometry())
        vol = torch.from_numpy(_vol(plan, seed)).cuda()
        y = torch.from_numpy(O.simulate_measurements(case)).cuda()
        want = B.vp_forward(plan, vol, y)       # also uploads the plan's tables
        torch.cuda.synchronize()
        out = torch.full(plan.blade_shape, float("nan"), dtype=torch.complex64, device="cuda")
        B.vp_forward_noalloc(plan, vol, out, y)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want.cpu().numpy())
        # without measurements, into the same output again
        want0 = B.vp_forward(plan, vol)
        B.vp_forward_noalloc(plan, vol, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want0.cpu().numpy())


def test_forward_noalloc_errors(gpu_lib):
    import torch
    from paper_2311_13177_amd import binding as B

    # a plan whose tables were never uploaded
    fresh = B.Plan.from_geometry(configs.small_case(n=40, n_spec=3, n_blades=2, lines=6, seed=23).geometry())
    vol = torch.zeros(fresh.volume_shape, dtype=torch.complex64, device="cuda")
    out = torch.zeros(fresh.blade_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(B.VPError) as ei:
        B.vp_forward_noalloc(fresh, vol, out)
    assert ei.value.status == B.VP_ERR_STATE
    # blade images beyond the 32 MiB scratch: 32 dynamic blades of 192^2 need 18.9 MB, 64
    # blades of 256^2 with two parts 67 MB
    g = configs.small_case(n=256, n_spec=2, n_time=2, n_blades=64, lines=8, seed=24).geometry()
    huge = B.Plan.from_geometry(g)
    hv = torch.zeros(huge.volume_shape, dtype=torch.complex64, device="cuda")
    ho = torch.zeros(huge.blade_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(B.VPError) as ei:
        B.vp_forward_noalloc(huge, hv, ho)
    assert ei.value.status == B.VP_ERR_UNSUPPORTED
