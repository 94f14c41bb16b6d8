"""Pins of the blade-aligned sampling oracle (non-uniform DFT and its gridding).

At 0 and 90 degrees a blade's lattice is the Cartesian mask, so the definition must
reproduce the unitary FFT there; the definition is its own adjoint's transpose; the
Kaiser-Bessel transform matches quadrature; the gridding approximation stays within
its bound of the definition and is exactly adjoint to itself; the lifted data term's
gradient passes central differences and reduces to the (pinned) Cartesian one.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle import nonuniform as N


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("theta", [0.0, math.pi / 2])
def test_axis_aligned_blades_are_the_cartesian_samples(theta):
    n, L = 16, 6
    rng = np.random.default_rng(1)
    img = _crandn(rng, n, n)
    kx, ky = N.blade_samples(n, theta, L)
    got = N.ndft_forward(img, kx, ky)
    spec = np.fft.fft2(img, norm="ortho")
    want = spec[np.rint(ky).astype(int) % n, np.rint(kx).astype(int) % n]
    assert np.allclose(got, want, atol=1e-12)
    # the same set of samples as the Cartesian mask of that blade
    mask = O.blade_mask(n, theta, L)
    pts = set(zip((np.rint(ky).astype(int) % n).ravel(), (np.rint(kx).astype(int) % n).ravel()))
    assert pts == set(zip(*np.nonzero(mask)))


def test_ndft_adjoint_and_kb_transform():
    n = 12
    rng = np.random.default_rng(2)
    kx, ky = N.blade_samples(n, 0.7, 5)
    f, s = _crandn(rng, n, n), _crandn(rng, *kx.shape)
    assert abs(np.vdot(s, N.ndft_forward(f, kx, ky)) - np.vdot(N.ndft_adjoint(s, kx, ky, n), f)) < 1e-10
    u = np.linspace(-N.KB_WIDTH / 2, N.KB_WIDTH / 2, 400001)
    for x in (0.0, 3.0, 11.5):
        q = np.trapezoid(N.kb_kernel(u) * np.cos(2 * np.pi * u * x / 24), u)
        assert math.isclose(float(N.kb_transform(x, 24)), q, rel_tol=1e-9)


@pytest.mark.parametrize("n,theta,L", [(16, 0.7, 6), (20, 2.3, 5), (15, 1.1, 4)])
def test_gridding_approximates_the_definition_and_is_self_adjoint(n, theta, L):
    rng = np.random.default_rng(n)
    kx, ky = N.blade_samples(n, theta, L)
    f, s = _crandn(rng, n, n), _crandn(rng, *kx.shape)
    fwd = N.nufft_forward(f, kx, ky)
    ref = N.ndft_forward(f, kx, ky)
    assert np.linalg.norm(fwd - ref) <= 1e-5 * np.linalg.norm(ref)
    adj = N.nufft_adjoint(s, kx, ky, n)
    aref = N.ndft_adjoint(s, kx, ky, n)
    assert np.linalg.norm(adj - aref) <= 1e-5 * np.linalg.norm(aref)
    lhs, rhs = np.vdot(s, fwd), np.vdot(adj, f)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _geom(n=12, s=3, angles=(0.0, 0.9, 2.2), lines=(4, 5, 3), t=1, times=None):
    return O.Geometry(n=n, n_spec=s, n_time=t, angle_rad=np.asarray(angles, dtype=np.float64),
                      lines=np.asarray(lines), blade_time=None if times is None else np.asarray(times),
                      spec_shift_px=np.linspace(-1.2, 1.9, s))


def test_lifted_gradient_central_difference():
    rng = np.random.default_rng(4)
    geom = _geom(t=2, times=(0.0, 0.4, 1.0))
    vol = _crandn(rng, 2, 3, 12, 12)
    y = [_crandn(rng, *N.blade_samples(12, float(a), int(L))[0].shape) for a, L in zip(geom.angle_rad, geom.lines)]
    g, val = N.gradient_nu(vol, geom, y)
    d = _crandn(rng, *vol.shape)
    h = 1e-3

    def f(v):
        return 0.5 * sum(float(np.sum(np.abs(s - yb) ** 2)) for s, yb in zip(N.forward_nu(v, geom), y))

    fd = (f(vol + h * d) - f(vol - h * d)) / (2 * h)
    assert math.isclose(fd, float(np.sum((np.conj(g) * d).real)), rel_tol=1e-9)
    assert math.isclose(val, f(vol), rel_tol=1e-12)


def test_axis_aligned_gradient_is_the_cartesian_gradient():
    rng = np.random.default_rng(5)
    n = 12
    geom = _geom(n=n, angles=(0.0, math.pi / 2), lines=(4, 6))
    vol = _crandn(rng, 1, 3, n, n)
    masks = O.blade_masks(geom)
    ygrid = masks * _crandn(rng, 2, n, n)
    y = []
    for b in range(2):
        kx, ky = N.blade_samples(n, float(geom.angle_rad[b]), int(geom.lines[b]))
        y.append(ygrid[b][np.rint(ky).astype(int) % n, np.rint(kx).astype(int) % n])
    g, val = N.gradient_nu(vol, geom, y)
    gc, vc = O.gradient(vol, geom, ygrid, 0.0, 1e-3)
    assert np.allclose(g, gc, atol=1e-11) and math.isclose(val, vc, rel_tol=1e-12)


def test_fit_on_axis_aligned_blades_is_the_cartesian_fit():
    # with blades at 0 and 90 degrees the blade-aligned fit is the Cartesian fit
    rng = np.random.default_rng(6)
    n = 12
    geom = _geom(n=n, angles=(0.0, math.pi / 2), lines=(4, 6))
    masks = O.blade_masks(geom)
    ygrid = masks * _crandn(rng, 2, n, n)
    y = []
    for b in range(2):
        kx, ky = N.blade_samples(n, float(geom.angle_rad[b]), int(geom.lines[b]))
        y.append(ygrid[b][np.rint(ky).astype(int) % n, np.rint(kx).astype(int) % n])
    a = N.reconstruct_nu(geom, y, 4, tv_weight=0.01, data_weight=1.5)
    c = O.reconstruct(geom, ygrid, 4, tv_weight=0.01, data_weight=1.5)
    assert np.allclose(a["vol"], c["vol"], atol=1e-10)
    assert math.isclose(a["final_loss"], c["final_loss"], rel_tol=1e-10)


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
def test_one_blade_fit_on_axis_aligned_blades_is_the_cartesian_one(schedule):
    rng = np.random.default_rng(7)
    n = 12
    geom = _geom(n=n, angles=(0.0, math.pi / 2), lines=(4, 6))
    ygrid = O.blade_masks(geom) * _crandn(rng, 2, n, n)
    y = []
    for b in range(2):
        kx, ky = N.blade_samples(n, float(geom.angle_rad[b]), int(geom.lines[b]))
        y.append(ygrid[b][np.rint(ky).astype(int) % n, np.rint(kx).astype(int) % n])
    a = N.reconstruct_nu(geom, y, 5, tv_weight=0.01, schedule=schedule, seed=9)
    c = O.reconstruct(geom, ygrid, 5, tv_weight=0.01, schedule=schedule, seed=9)
    assert np.allclose(a["vol"], c["vol"], atol=1e-10)
    assert math.isclose(a["final_loss"], c["final_loss"], rel_tol=1e-10)
