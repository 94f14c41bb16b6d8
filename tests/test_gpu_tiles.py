"""Tile shapes and the autotuner on the GPU.

A tile shape only changes how the projection, gather and update work is cut into
work items (and whether the update runs fused into the gather or as its own pass);
every voxel's arithmetic, and its order, stays the same. So every shape must give
the same bits, alone, batched with slices of another shape, and through the
operators, and the shape the tuner records must be one of them.
"""

import numpy as np
import pytest

import oracle as O
from parity import assert_close
from synth import configs

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 1, 2, 1, 0), (2, 4, 2, 8, 0), (4, 1, 4, 4, 0), (8, 2, 4, 2, 0),
    (1, 8, 2, 2, 2), (4, 2, 2, 4, 4), (8, 1, 4, 1, 8),
    # eight waves per gather or projection item
    (2, 1, 2, 4, 0, 8), (4, 2, 4, 1, 0, 8), (2, 2, 2, 8, 0, 8), (1, 1, 4, 2, 2, 8),
    (4, 1, 2, 4, 0, 8, 8), (1, 2, 2, 2, 0, 4, 8), (8, 1, 4, 1, 4, 8, 8),
    # every part of a knot resident in LDS, each bin gathered and updated in turn
    (2, 1, 2, 4, 0, 4, 4, 1), (4, 2, 4, 2, 0, 8, 4, 1), (1, 1, 2, 8, 0, 8, 8, 1), (2, 2, 4, 1, 0, 4, 4, 1),
    (8, 1, 2, 1, 0, 8, 4, 1),
    # twelve-row projection tiles
    (12, 1, 2, 2, 0, 4, 8), (12, 1, 4, 8, 0, 8, 4, 1),
]

CASES = {
    "static_80": dict(n=80, n_spec=5, n_blades=3, lines=10, f=3.0),
    "static_90_s13": dict(n=90, n_spec=13, n_blades=9, lines=9),
    "dynamic_40": dict(n=40, n_spec=5, n_time=3, n_blades=6, lines=8),
    "dynamic_72": dict(n=72, n_spec=6, n_time=5, n_blades=11, lines=10, f=2.5),
}


def _problem(B, name, steps):
    case = configs.small_case(**CASES[name])
    plan = B.Plan.from_geometry(case.geometry())
    y = O.simulate_measurements(case)
    return case, plan, y


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("vol", "proj", "water", "fat")) and \
        a["final_loss"] == b["final_loss"]


@pytest.mark.parametrize("name", sorted(CASES))
def test_every_shape_gives_the_same_bits(gpu_lib, name):
    from paper_2311_13177_amd import binding as B

    case, plan, y = _problem(B, name, 9)
    for opt in (B.VP_OPT_ADAM, B.VP_OPT_GD):
        ref = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=9, optimizer=opt))
        for sh in SHAPES:
            got = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=9, optimizer=opt, tiles=sh))
            assert _same(got, ref), (opt, sh)
    # and the common result is the method's (GD: linear dynamics, the operator tolerance)
    geom = O.Geometry.from_dict(case.geometry())
    want = O.reconstruct(geom, y, 9, optimizer="gd")
    assert_close(ref["vol"], want["vol"], 1e-4)


def test_batch_of_different_shapes_equals_solo(gpu_lib):
    from paper_2311_13177_amd import binding as B

    probs = [_problem(B, name, 0) for name in sorted(CASES)]
    opts = [B.vp_options_default(n_steps=7 + i, tiles=SHAPES[(2 * i + 1) % len(SHAPES)])
            for i in range(len(probs))]
    solo = [B.vp_reconstruct(p, y, o) for (_, p, y), o in zip(probs, opts)]
    got = B.vp_batch_reconstruct([p for _, p, _ in probs], [y for _, _, y in probs], opts)
    for g, s in zip(got, solo):
        assert g["status"] == 0 and _same(g, s)


def test_tuner_records_a_shape_that_sessions_and_operators_use(gpu_lib):
    import torch
    from paper_2311_13177_amd import binding as B

    case, plan, y = _problem(B, "dynamic_72", 0)
    before = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=6))
    tuned = plan.tune(B.vp_options_default())
    pr, pp, gr, gb, ub, gw, pw, res = tuned
    assert pr in (1, 2, 4, 8) and pp in (1, 2, 4, 8) and pr * pp <= 16 and pw in (4, 8)
    assert gr in (2, 4) and gb in (1, 2, 4, 8) and gr * gb <= 16 and ub in (0, 2, 4, 8) and gw in (4, 8)
    assert res in (0, 1) and not (res and ub)
    assert plan.tiles(B.vp_options_default()) == tuned
    # a second plan of the same sizes picks the recorded shape up
    again = B.Plan.from_geometry(case.geometry())
    assert again.tiles(B.vp_options_default()) == tuned
    after = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=6))
    assert _same(after, before)
    # the operators follow the tuned layout and still match the oracle
    vol = np.random.default_rng(3).standard_normal(plan.volume_shape).astype(np.complex64)
    d_vol = torch.from_numpy(vol).to("cuda")
    d_out = torch.empty(plan.blade_shape, dtype=torch.complex64, device="cuda")
    B.vp_forward(plan, d_vol, None, d_out)
    want = O.forward(vol.astype(np.complex128), O.Geometry.from_dict(case.geometry()))
    got = d_out.cpu().numpy()
    assert_close(got, want, 1e-4)


def test_autotune_option_tunes_once(gpu_lib):
    from paper_2311_13177_amd import binding as B

    case, plan, y = _problem(B, "static_90_s13", 0)
    o = B.vp_options_default(n_steps=5, autotune=1)
    r1 = B.vp_reconstruct(plan, y, o)
    shape = plan.tiles(o)
    r2 = B.vp_reconstruct(plan, y, B.vp_options_default(n_steps=5))
    assert plan.tiles(B.vp_options_default()) == shape
    assert _same(r1, r2)


def test_compiled_adam_tv_epilogue_equals_the_generic_one(gpu_lib):
    # alone, Adam with TV and no L1 runs the epilogue compiled for it; batched with a slice
    # that needs run-time options (GD, or L1) the whole group takes the generic epilogue
    from paper_2311_13177_amd import binding as B

    probs = [_problem(B, name, 0) for name in ("static_80", "dynamic_72", "dynamic_40")]
    opts = [B.vp_options_default(n_steps=8), B.vp_options_default(n_steps=8, tiles=(2, 2, 2, 4, 2)),
            B.vp_options_default(n_steps=8, l1_weight=1e-4)]
    solo = [B.vp_reconstruct(p, y, o) for (_, p, y), o in zip(probs, opts)]
    got = B.vp_batch_reconstruct([p for _, p, _ in probs], [y for _, _, y in probs], opts)
    for g, s in zip(got, solo):
        assert g["status"] == 0 and _same(g, s)
