"""Baselines and PSNR on the GPU (Section 6) against the oracle, through the C ABI.

The baseline is an average and an inverse DFT in FP32 against the FP64 oracle, so it
takes the operator tolerance (1e-4 relative over all frames). PSNR accumulates in FP64
from the FP32 inputs that the oracle up-casts, so it agrees to about 1e-12.
"""

import math

import numpy as np
import pytest

import oracle as O
from parity import both_bounds
from synth import configs

pytestmark = pytest.mark.gpu

CASES = {
    # generic and specialised transform lengths, static and dynamic, ragged tails
    "static_80": dict(n=80, n_spec=5, n_blades=3, lines=10, f=3.0),
    "static_64": dict(n=64, n_spec=4, n_blades=5, lines=16),
    "dynamic_72": dict(n=72, n_spec=6, n_time=5, n_blades=11, lines=10, f=2.5),
    "dynamic_192": dict(n=192, n_spec=4, n_time=4, n_blades=8, lines=24, f=3.0),
}


def _rel(a, b):
    # both bounds of tests/parity.py in one number: a tolerance on it bounds the relative
    # L2 error and the largest element error relative to the largest reference magnitude
    return both_bounds(a, b)


def _setup(name):
    import torch
    from paper_2311_13177_amd import binding as B

    case = configs.small_case(**CASES[name])
    plan = B.Plan.from_geometry(case.geometry())
    y = O.simulate_measurements(case)
    masks = O.blade_masks(O.Geometry.from_dict(case.geometry()))
    return B, case, plan, y, masks, torch.from_numpy(y).to("cuda")


@pytest.mark.parametrize("name", sorted(CASES))
def test_baseline_matches_oracle(gpu_lib, name):
    B, case, plan, y, masks, d_y = _setup(name)
    nb = y.shape[0]
    yy = y.astype(np.complex128)
    # static: every blade, the last frame
    got = B.vp_baseline(plan, d_y).cpu().numpy()
    want = O.coverage_baseline(yy, masks)
    assert got.shape == (1,) + want.shape and _rel(got[0], want) <= 1e-4
    # windows of 1, 5 and more than B blades, over every frame and over a ragged range
    for window in (1, 5, nb + 3):
        frames = O.window_baseline(yy, masks, window)
        got = B.vp_baseline(plan, d_y, window=window, first_frame=0, n_frames=nb).cpu().numpy()
        assert _rel(got, frames) <= 1e-4, window
        f0, nf = min(2, nb - 1), max(1, nb - 3)
        part = B.vp_baseline(plan, d_y, window=window, first_frame=f0, n_frames=nf).cpu().numpy()
        np.testing.assert_array_equal(part, got[f0:f0 + nf])


def test_baseline_argument_errors(gpu_lib):
    import torch

    B, case, plan, y, masks, d_y = _setup("static_80")
    nb = y.shape[0]
    lib = B.lib()
    out = torch.empty((nb,) + y.shape[1:], dtype=torch.complex64, device="cuda")
    s = B._stream(None)
    from ctypes import c_void_p

    for first, nf in ((-1, 1), (0, nb + 1), (nb - 1, 2), (0, -1)):
        assert lib.vp_baseline(plan.handle, c_void_p(d_y.data_ptr()), 0, first, nf,
                               c_void_p(out.data_ptr()), s) == -1, (first, nf)
    # the output may not overlap the measurements
    assert lib.vp_baseline(plan.handle, c_void_p(d_y.data_ptr()), 0, 0, 1,
                           c_void_p(d_y.data_ptr() + 8), s) == -1
    assert lib.vp_baseline(plan.handle, c_void_p(d_y.data_ptr()), 0, 0, 0, None, s) == 0


def test_psnr_matches_oracle(gpu_lib):
    import torch
    from paper_2311_13177_amd import binding as B

    rng = np.random.default_rng(61)
    shape = (3, 37, 53)
    truth = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    image = (truth + 0.05 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)
    image[2] = truth[2] * np.complex64(1j)  # equal magnitudes: +inf
    d_t, d_i = torch.from_numpy(truth).to("cuda"), torch.from_numpy(image).to("cuda")
    p, mse, peak = (x.cpu().numpy() for x in B.vp_psnr(d_i, d_t))
    for k in range(3):
        want = O.psnr(image[k].astype(np.complex128), truth[k].astype(np.complex128))
        if math.isinf(want):
            assert math.isinf(p[k]) and mse[k] == 0.0
        else:
            assert math.isclose(p[k], want, rel_tol=1e-12)
        assert math.isclose(peak[k], np.abs(truth[k].astype(np.complex128)).max(), rel_tol=1e-15)
    # one image, and deterministic
    p1, _, _ = B.vp_psnr(d_i[0], d_t[0])
    assert p1.cpu().numpy()[0] == p[0]


def test_reconstruction_beats_the_baseline_on_a_fat_shifted_phantom(gpu_lib):
    # context, in the spirit of Table 1: with a fat shift of 8 px the lifted reconstruction
    # removes chemical shift that the baseline keeps (the oracle gives 28.9 dB against
    # 27.3 dB for this case, lr 3e-2, TV weight 1e-2, 200 steps)
    import torch
    from paper_2311_13177_amd import binding as B

    case = configs.small_case(n=64, n_spec=8, n_blades=5, lines=16, f=8.0, seed=11)
    plan = B.Plan.from_geometry(case.geometry())
    y = O.simulate_measurements(case)
    w, f = case.layers_at(0.0)
    truth = torch.from_numpy((w + f).astype(np.complex64)).to("cuda")
    base = B.vp_baseline(plan, torch.from_numpy(y).to("cuda"))[0]
    r = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=200, lr=3e-2, tv_weight=1e-2))
    ours = torch.from_numpy(r["proj"][0].astype(np.complex64)).to("cuda")
    p_base = B.vp_psnr(base, truth)[0].item()
    p_ours = B.vp_psnr(ours, truth)[0].item()
    assert p_ours > p_base + 1.0, (p_ours, p_base)


def test_dynamic_workload_beats_its_baseline(gpu_lib):
    # context on a benchmark workload with its own settings: the dynamic 192^2 scan (S 32,
    # T 16, 32 golden-angle blades, lr 1e-2, TV 1e-3, 800 Adam steps); the baseline is the
    # coverage-weighted average of each frame's five most recent blades, which lags the
    # motion. PSNR on magnitudes, averaged over frames (knot frames at the knot times for
    # the fit, blade frames at the blade times for the baseline).
    import torch
    from paper_2311_13177_amd import binding as B

    case = configs.dynamic_192()
    plan = B.Plan.from_geometry(case.geometry())
    y = O.simulate_measurements(case)

    def truth(tau):
        w, f = case.layers_at(float(tau))
        return (w + f).astype(np.complex64)

    r = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=case.n_steps, lr=case.lr, tv_weight=case.tv_weight))
    t_knots = torch.from_numpy(np.stack([truth(k / (case.n_time - 1)) for k in range(case.n_time)])).to("cuda")
    ours = B.vp_psnr(torch.from_numpy(r["proj"].astype(np.complex64)).to("cuda"), t_knots)[0].cpu().numpy()
    base = B.vp_baseline(plan, torch.from_numpy(y).to("cuda"), window=5, first_frame=0, n_frames=case.n_blades)
    t_blades = torch.from_numpy(np.stack([truth(t) for t in case.blade_time])).to("cuda")
    theirs = B.vp_psnr(base, t_blades)[0].cpu().numpy()
    print(f"dynamic_192: fit {ours.mean():.2f} dB, five-blade baseline {theirs.mean():.2f} dB")
    assert ours.mean() > theirs.mean() + 1.0
