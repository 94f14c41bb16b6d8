"""Host-side checks of the C ABI: exports, plan tables against the oracle, validation.

These run without a GPU: vp_plan_create and its accessors touch no device.
"""

import math
import os
import re

import numpy as np
import pytest

import oracle as O
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2311_13177_amd import binding

    binding.lib()
    return binding


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "vp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:vp_status|const char\*)\s+(vp_\w+)\s*\(", text, flags=re.M)))


def test_header_and_library_exports_agree(B):
    declared = _declared_functions()
    assert len(declared) >= 30
    lib = B.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(B.exported_names()) == declared


def _plan(B, case):
    return B.Plan.from_geometry(case.geometry())


@pytest.mark.parametrize("name", ["static_64", "static_256", "dynamic_192"])
def test_masks_match_oracle_bit_for_bit(B, name):
    case = configs.CONFIGS[name]()
    plan = _plan(B, case)
    geom = O.Geometry.from_dict(case.geometry())
    want = O.blade_masks(geom)
    got = plan.masks()
    assert np.array_equal(got, want)
    # the paper's blade widths: L lines along each of n readout samples on axis-aligned blades
    for b in range(case.n_blades):
        if abs(math.sin(case.angle_rad[b])) < 1e-12 or abs(math.cos(case.angle_rad[b])) < 1e-12:
            assert got[b].sum() == case.lines[b] * case.n


def test_shear_table_matches_oracle_taps(B):
    case = configs.static_256()
    plan = _plan(B, case)
    for b in range(case.n_blades):
        for s in range(case.n_spec):
            d = O.displacement(float(case.angle_rad[b]), float(case.spec_shift_px[s]))
            tp = O.taps(d)
            ox, oy, fx, fy = plan.shear(b, s)
            assert (oy, ox) == (tp[0][0], tp[0][1])
            assert abs(fx - (-d[0] - ox)) < 1e-7 and abs(fy - (-d[1] - oy)) < 1e-7


def test_knot_weights_match_oracle(B):
    case = configs.dynamic_192()
    plan = _plan(B, case)
    for b in range(case.n_blades):
        k, a = plan.knot(b)
        k0, a0 = O.knot_weights(float(case.blade_time[b]), case.n_time)
        assert k == k0 and abs(a - a0) < 1e-7


def _geom(**kw):
    g = dict(n=16, n_spec=4, n_time=1, angle_rad=[0.0, 1.0], lines=[4, 4], blade_time=None,
             spec_shift_px=[0.0, 0.5, 1.0, 1.5])
    g.update(kw)
    return g


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), -1),
    (dict(n_spec=0, spec_shift_px=[]), -1),
    (dict(lines=[0, 4]), -1),
    (dict(lines=[4, 17]), -1),
    (dict(angle_rad=[0.0, float("nan")]), -1),
    (dict(spec_shift_px=[0.0, float("inf"), 1.0, 1.5]), -1),
    (dict(n_time=2, blade_time=None), -1),
    (dict(blade_time=[0.0, 0.5]), -1),
    (dict(n_time=2, blade_time=[0.0, 1.5]), -1),
    (dict(n=14), -2),
    (dict(n=1024), -2),
    (dict(spec_shift_px=[0.0, 0.5, 1.0, 16.5]), -2),
])
def test_plan_validation_errors(B, kw, code):
    with pytest.raises(B.VPError) as ei:
        B.Plan.from_geometry(_geom(**kw))
    assert ei.value.status == code
    assert B.lib().vp_last_error().decode() != ""


def test_supported_sizes(B):
    for n in (1, 2, 3, 5, 6, 48, 60, 64, 96, 120, 128, 192, 240, 256, 320, 384, 480, 500, 512):
        B.Plan.from_geometry(_geom(n=n, lines=[1, 1]))


def test_device_bytes_formula(B):
    case = configs.static_256()
    plan = _plan(B, case)
    opts = B.vp_options_default()
    got = plan.device_bytes(opts)
    vox = 32 * 256 * 256 * 8
    blade = 12 * 256 * 256 * 8
    # volume ping-pong + Adam moments + data gradient + blade work + measurements
    assert got >= 5 * vox + 2 * blade
    assert got < 5 * vox + 2 * blade + 4 * 1024 * 1024
    gd = B.vp_options_default(optimizer=B.VP_OPT_GD)
    assert plan.device_bytes(gd) == got - 2 * vox


def test_status_strings(B):
    lib = B.lib()
    for code in range(0, -11, -1):
        assert lib.vp_status_string(code).decode()
    assert lib.vp_status_string(-99).decode() == "unknown status"


def test_oracle_does_not_import_product():
    import ast

    for dirpath, _, files in os.walk(os.path.join(ROOT, "oracle")):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, (ast.Import, ast.ImportFrom)):
                        mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                        for m in mods:
                            assert not m.startswith("paper_2311_13177_amd"), (f, m)


def test_product_does_not_import_oracle():
    import ast

    pkg = os.path.join(ROOT, "paper_2311_13177_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, (ast.Import, ast.ImportFrom)):
                        mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                        for m in mods:
                            assert not m.startswith("oracle"), (f, m)
                            assert not m.startswith("synth"), (f, m)


def _tiles_ok(t):
    pr, pp, gr, gb, ub, gw, pw, res = t
    return (pr in (1, 2, 4, 8) and pp in (1, 2, 4, 8) and pr * pp <= 16 and gr in (2, 4)
            and gb in (1, 2, 4, 8) and gr * gb <= 16 and ub in (0, 2, 4, 8) and gw in (4, 8) and pw in (4, 8)
            and res in (0, 1) and not (res and ub))


@pytest.mark.parametrize("name", ["static_64", "static_256", "dynamic_192"])
def test_builtin_tile_shape_without_a_device(B, name):
    """Without tuning, the shape comes from the plan alone (no device is touched)."""
    plan = _plan(B, configs.CONFIGS[name]())
    t = plan.tiles(B.vp_options_default())
    assert _tiles_ok(t)
    # an explicit shape is taken as given
    assert plan.tiles(B.vp_options_default(tiles=(8, 1, 4, 4, 8))) == (8, 1, 4, 4, 8, 4, 4, 0)
    assert plan.tiles(B.vp_options_default(tiles=(2, 2, 2, 4, 0, 8))) == (2, 2, 2, 4, 0, 8, 4, 0)
    assert plan.tiles(B.vp_options_default(tiles=(4, 1, 2, 4, 0, 0, 8))) == (4, 1, 2, 4, 0, 4, 8, 0)


@pytest.mark.parametrize("name,fits", [("static_64", True), ("dynamic_192", True), ("static_256", False)])
def test_resident_gather_shape_where_the_parts_fit(B, name, fits):
    """The resident-parts gather stages every part of a knot at once: a plan takes it when
    the largest knot's parts fit 64 KiB of LDS (five parts of at most 666 elements in the
    dynamic 192^2 workload) and refuses it otherwise (twelve parts of 836 elements, 80 KiB,
    at 256^2), and never with a separate update pass."""
    plan = _plan(B, configs.CONFIGS[name]())
    shape = (2, 1, 2, 8, 0, 4, 4, 1)
    if fits:
        assert plan.tiles(B.vp_options_default(tiles=shape)) == shape
    else:
        with pytest.raises(B.VPError) as ei:
            plan.tiles(B.vp_options_default(tiles=shape))
        assert ei.value.status == B.VP_ERR_UNSUPPORTED
    with pytest.raises(B.VPError) as ei:
        plan.tiles(B.vp_options_default(tiles=(2, 1, 2, 8, 4, 4, 4, 1)))
    assert ei.value.status == B.VP_ERR_UNSUPPORTED


@pytest.mark.parametrize("tiles", [(3, 1, 2, 1, 0), (8, 4, 2, 1, 0), (2, 1, 1, 1, 0), (2, 1, 4, 8, 0),
                                   (2, 1, 2, 16, 0), (2, 1, 2, 1, 3), (0, 0, 0, 0, 4), (2, 1, 2, 1, 0, 2),
                                   (2, 1, 2, 1, 0, 16), (0, 0, 0, 0, 0, 8), (2, 1, 2, 1, 0, 4, 6),
                                   (0, 0, 0, 0, 0, 0, 8), (2, 1, 2, 1, 0, 4, 4, 2), (2, 1, 2, 1, 2, 4, 4, 1)])
def test_uncompiled_tile_shapes_are_rejected(B, tiles):
    plan = _plan(B, configs.static_64())
    with pytest.raises(B.VPError) as ei:
        plan.tiles(B.vp_options_default(tiles=tiles))
    assert ei.value.status == B.VP_ERR_UNSUPPORTED


def test_kplanes_param_count_and_model_checks():
    import ctypes

    from oracle import kplanes as K
    from paper_2311_13177_amd import binding as B

    case = configs.small_case(n=40, n_spec=5, n_time=3, n_blades=4)
    plan = B.Plan.from_geometry(case.geometry())
    m = B.vp_kplanes.make(8, 6, (40, 20), 1e-3, 1e-2, 1e-3, 1e-3)
    _, _, total = K.layout(5, K.KPConfig(features=8, time_res=6, spatial_res=(40, 20)))
    assert B.kplanes_param_count(plan, m) == total
    out = ctypes.c_int64()
    for bad in (B.vp_kplanes.make(3, 6, (40,)), B.vp_kplanes.make(8, 0, (40,)), B.vp_kplanes.make(8, 6, (41,)),
                B.vp_kplanes.make(8, 6, (40,), eps=0.0), B.vp_kplanes.make(8, 6, (40,), tv_weight=float("inf"))):
        assert B.lib().vp_kplanes_param_count(plan.handle, ctypes.byref(bad), ctypes.byref(out)) == B.VP_ERR_ARG
    three = B.vp_kplanes.make(8, 6, (40, 20))
    three.n_scales = 3
    assert B.lib().vp_kplanes_param_count(plan.handle, ctypes.byref(three), ctypes.byref(out)) == B.VP_ERR_ARG
