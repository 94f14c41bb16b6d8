"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-force
DFT, the Fourier shift theorem the paper's Section 3 rests on, a hand-derived
mask, exact Adam arithmetic, closed-form gradient-descent trajectories, adjoint
identities and finite differences.
"""

import math
import os

import numpy as np
import pytest

import oracle as O
from synth import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geom(n=16, s=3, t=1, angles=(0.0, 0.7, 2.0), lines=(4, 6, 5), times=None, shifts=None):
    angles = np.asarray(angles, dtype=np.float64)
    if shifts is None:
        shifts = np.linspace(-1.3, 2.2, s)
    return O.Geometry(n=n, n_spec=s, n_time=t, angle_rad=angles, lines=np.asarray(lines),
                      blade_time=None if times is None else np.asarray(times, dtype=np.float64),
                      spec_shift_px=np.asarray(shifts, dtype=np.float64))


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ------------------------------------------------------------------ DFT (Section 4.2 "Blur")

@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 12])
def test_unitary_dft_matches_brute_force(n):
    rng = np.random.default_rng(n)
    x = _crandn(rng, n, n)
    j = np.arange(n)
    f = np.exp(-2j * math.pi * np.outer(j, j) / n)
    brute = f @ x @ f.T / n
    assert np.allclose(np.fft.fft2(x, norm="ortho"), brute, rtol=0, atol=1e-13)
    # the signed-frequency labelling of unshifted storage gives the same exponentials
    k = O.signed_freq(n)
    f2 = np.exp(-2j * math.pi * np.outer(k, j) / n)
    assert np.allclose(f, f2, atol=1e-12)
    # inverse and Parseval
    assert np.allclose(np.fft.ifft2(np.fft.fft2(x, norm="ortho"), norm="ortho"), x, atol=1e-13)
    assert math.isclose(np.linalg.norm(np.fft.fft2(x, norm="ortho")), np.linalg.norm(x), rel_tol=1e-13)


def test_signed_freq_values():
    assert list(O.signed_freq(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(O.signed_freq(5)) == [0, 1, 2, -2, -1]


# ------------------------------------------------------------------ masks

def _read_mask_fixture():
    blades = []
    with open(os.path.join(GOLDEN, "mask_n8_l2.txt")) as fh:
        cur = None
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "blade":
                cur = dict(theta=float(parts[1]), n=int(parts[2]), lines=int(parts[3]),
                           count=int(parts[4]), pts=[])
                blades.append(cur)
            else:
                cur["pts"].append((int(parts[0]), int(parts[1])))
    return blades


def test_mask_matches_hand_derivation():
    for bl in _read_mask_fixture():
        n = bl["n"]
        want = np.zeros((n, n), dtype=bool)
        for ky, kx in bl["pts"]:
            want[ky % n, kx % n] = True
        assert want.sum() == bl["count"]
        got = O.blade_mask(n, math.radians(bl["theta"]), bl["lines"])
        assert np.array_equal(got, want), bl["theta"]


@pytest.mark.parametrize("n,lines", [(64, 16), (256, 32), (192, 24), (48, 12)])
def test_mask_axis_aligned_counts(n, lines):
    for deg in (0.0, 90.0):
        m = O.blade_mask(n, math.radians(deg), lines)
        assert int(m.sum()) == lines * n


def test_mask_rotation_by_180_is_point_mirror():
    # the blade's support is symmetric about the origin up to the half-open edges:
    # theta and theta + pi give the mirrored set k -> -k
    n, lines = 32, 8
    for deg in (10.0, 36.0, 72.0):
        a = O.blade_mask(n, math.radians(deg), lines)
        b = O.blade_mask(n, math.radians(deg + 180.0), lines)
        k = O.signed_freq(n)
        # mirror index map j -> -j mod n
        idx = (-np.arange(n)) % n
        mirrored = a[np.ix_(idx, idx)]
        # interior samples (away from the |r| = n/2 and |q| = L/2 edges) agree
        ky, kx = np.meshgrid(k, k, indexing="ij")
        c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
        r = kx * c + ky * s
        q = -kx * s + ky * c
        interior = (np.abs(r) < n / 2 - 1) & (np.abs(q) < lines / 2 - 1)
        assert np.array_equal(mirrored[interior], b[interior])


# ------------------------------------------------------------------ shear vs physics (Section 3)

def test_integer_shift_is_linear_phase():
    # Section 3: a single frequency offset is a linear phase along the blade, i.e. a
    # translation of the image. For an integer displacement the bilinear shear is an
    # exact translation, so the blade's k-space is the bin's DFT times exp(-2 pi i k.d/n).
    n = 32
    rng = np.random.default_rng(1)
    img = np.zeros((n, n), dtype=np.complex128)
    img[10:20, 9:21] = _crandn(rng, 10, 12)
    k = O.signed_freq(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    for theta, delta in ((0.0, 3.0), (math.pi / 2, -2.0), (math.pi / 4, 2 * math.sqrt(2.0)), (math.pi, 1.0)):
        dx, dy = O.displacement(theta, delta)
        dxi, dyi = round(dx), round(dy)
        assert abs(dx - dxi) < 1e-12 and abs(dy - dyi) < 1e-12
        shifted = O.shear(img, (float(dxi), float(dyi)))
        phase = np.exp(-2j * math.pi * (kx * dxi + ky * dyi) / n)
        assert np.allclose(np.fft.fft2(shifted, norm="ortho"), phase * np.fft.fft2(img, norm="ortho"),
                           atol=1e-12)


def test_fractional_shift_transfer_function():
    # A bilinear shift of an image whose support stays inside the grid is a filter with
    # the separable transfer function H_x H_y,
    # H_x = exp(2 pi i k_x o_x / n) ((1 - f_x) + f_x exp(2 pi i k_x / n)),  o = floor(-d), f = -d - o.
    n = 24
    rng = np.random.default_rng(2)
    img = np.zeros((n, n), dtype=np.complex128)
    img[6:17, 7:18] = _crandn(rng, 11, 11)
    k = O.signed_freq(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    for d in ((0.3, -1.7), (-2.25, 0.5), (1.0, 0.0), (3.9, 2.1)):
        o = (math.floor(-d[0]), math.floor(-d[1]))
        f = (-d[0] - o[0], -d[1] - o[1])
        hx = np.exp(2j * math.pi * kx * o[0] / n) * ((1 - f[0]) + f[0] * np.exp(2j * math.pi * kx / n))
        hy = np.exp(2j * math.pi * ky * o[1] / n) * ((1 - f[1]) + f[1] * np.exp(2j * math.pi * ky / n))
        lhs = np.fft.fft2(O.shear(img, d), norm="ortho")
        assert np.allclose(lhs, hx * hy * np.fft.fft2(img, norm="ortho"), atol=1e-12)


def test_point_source_moves_by_displacement():
    # Section 4.2: material at spectral height delta lands displaced by delta along the
    # blade direction. The bilinear image of a point keeps its mass and its centroid moves
    # by exactly d.
    n = 32
    x0, y0 = 13, 17
    img = np.zeros((n, n), dtype=np.complex128)
    img[y0, x0] = 1.0
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for theta in (0.3, 1.1, 2.5):
        for delta in (-2.4, 0.6, 3.3):
            dx, dy = O.displacement(theta, delta)
            out = O.shear(img, (dx, dy)).real
            assert math.isclose(out.sum(), 1.0, rel_tol=1e-13)
            assert math.isclose((out * xx).sum(), x0 + dx, abs_tol=1e-12)
            assert math.isclose((out * yy).sum(), y0 + dy, abs_tol=1e-12)


def test_shear_zero_outside_grid():
    n = 8
    img = np.ones((n, n), dtype=np.complex128)
    out = O.shear(img, (2.0, 0.0))   # material moves right by 2: columns 0, 1 read outside
    assert np.all(out[:, :2] == 0) and np.all(out[:, 2:] == 1)


# ------------------------------------------------------------------ adjoint identities

def test_shear_transpose_is_negated_shear():
    rng = np.random.default_rng(3)
    g = _crandn(rng, 20, 20)
    for d in ((0.3, -1.7), (-2.25, 0.5), (1.0, 0.0), (-0.0, 4.75), (5.5, -3.125)):
        a = O.shear_transpose(g, d)
        b = O.shear(g, (-d[0], -d[1]))
        assert np.allclose(a, b, atol=1e-14)


def test_shear_dot_product():
    rng = np.random.default_rng(4)
    x = _crandn(rng, 18, 18)
    y = _crandn(rng, 18, 18)
    for d in ((0.3, -1.7), (2.6, 1.2)):
        lhs = np.vdot(y, O.shear(x, d))
        rhs = np.vdot(O.shear_transpose(y, d), x)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("t,times", [(1, None), (3, (0.0, 0.45, 1.0))])
def test_operator_dot_product(t, times):
    geom = _geom(n=12, s=3, t=t, times=times)
    rng = np.random.default_rng(5)
    v = _crandn(rng, t, 3, 12, 12)
    k = _crandn(rng, 3, 12, 12)
    lhs = np.vdot(k, O.forward(v, geom))
    rhs = np.vdot(O.adjoint(k, geom), v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ gradients

def _fd_check(f, grad, v, rng, h, tol):
    for _ in range(3):
        d = _crandn(rng, *v.shape)
        fd = (f(v + h * d) - f(v - h * d)) / (2 * h)
        an = float(np.real(np.vdot(grad, d)))
        assert abs(fd - an) <= tol * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("t,times", [(1, None), (2, (0.1, 0.5, 0.95))])
def test_data_gradient_central_difference(t, times):
    geom = _geom(n=10, s=3, t=t, times=times)
    rng = np.random.default_rng(6)
    v = _crandn(rng, t, 3, 10, 10)
    y = _crandn(rng, 3, 10, 10)
    g, _ = O.gradient(v, geom, y, 0.0, 1e-3)
    # the data term is quadratic: the central difference is exact up to rounding
    _fd_check(lambda w: O.data_loss(O.residual(w, geom, y)), g, v, rng, h=0.5, tol=1e-9)


def test_tv_and_l1_gradients_central_difference():
    rng = np.random.default_rng(7)
    v = _crandn(rng, 2, 3, 6, 6)
    _fd_check(lambda w: O.tv_value(w, 1e-1), O.tv_grad(v, 1e-1), v, rng, h=1e-5, tol=1e-6)
    _fd_check(lambda w: O.l1_value(w, 1e-1), O.l1_grad(v, 1e-1), v, rng, h=1e-5, tol=1e-6)


def test_tv_closed_forms():
    eps = 1e-3
    assert O.tv_value(np.full((2, 3, 5, 5), 0.7 - 0.2j), eps) == 0.0
    # a single step of complex height h between columns 2 and 3 of a 1x1x4x6 volume:
    # four rows of one jump each, every other difference zero
    v = np.zeros((1, 1, 4, 6), dtype=np.complex128)
    h = 0.3 + 0.4j
    v[..., 3:] = h
    want = 4 * (math.sqrt(abs(h) ** 2 + eps ** 2) - eps)
    assert math.isclose(O.tv_value(v, eps), want, rel_tol=1e-14)
    g = O.tv_grad(v, eps)
    w = h / math.sqrt(abs(h) ** 2 + eps ** 2)
    assert np.allclose(g[..., 2], -w) and np.allclose(g[..., 3], w)
    assert np.allclose(g[..., [0, 1, 4, 5]], 0)


# ------------------------------------------------------------------ optimiser

def test_adam_matches_exact_arithmetic():
    rows = []
    with open(os.path.join(GOLDEN, "adam_two_params.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()[1:]])
    grads = [1 - 1j, 3 + 0.5j, -2 + 0.25j]
    vol = np.zeros(1, dtype=np.complex128)
    m = np.zeros((1, 2))
    v = np.zeros((1, 2))
    for t, (g, want) in enumerate(zip(grads, rows), 1):
        vol, m, v = O.adam_update(vol, np.array([g]), m, v, t, 0.1, 0.9, 0.999, 1e-8)
        assert abs(vol[0].real - want[0]) < 1e-15 and abs(vol[0].imag - want[1]) < 1e-15


def test_adam_first_step_from_zero():
    rng = np.random.default_rng(8)
    g = _crandn(rng, 50)
    vol, _, _ = O.adam_update(np.zeros(50, complex), g, np.zeros((50, 2)), np.zeros((50, 2)), 1,
                              0.01, 0.9, 0.999, 1e-8)
    want = -0.01 * (g.real / (np.abs(g.real) + 1e-8) + 1j * g.imag / (np.abs(g.imag) + 1e-8))
    assert np.allclose(vol, want, rtol=1e-14, atol=0)


def test_adam_matches_torch_cpu_fp64():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    p0 = _crandn(rng, 7)
    p = torch.tensor(np.stack([p0.real, p0.imag], -1), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    vol = p0.copy()
    m = np.zeros((7, 2))
    v = np.zeros((7, 2))
    for t in range(1, 6):
        g = _crandn(rng, 7)
        opt.zero_grad()
        p.grad = torch.tensor(np.stack([g.real, g.imag], -1), dtype=torch.float64)
        opt.step()
        vol, m, v = O.adam_update(vol, g, m, v, t, 0.05, 0.9, 0.999, 1e-8)
    got = p.detach().numpy()
    assert np.allclose(got[:, 0], vol.real, rtol=1e-13, atol=1e-15)
    assert np.allclose(got[:, 1], vol.imag, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------ zero off-resonance closed form

def test_zero_offresonance_gd_reduces_to_multiblade_dft_fit():
    # With every bin unshifted the lifted model collapses to U = sum_s V_s seen by every
    # blade; gradient descent from zero with step eta gives, per k-space sample,
    #   DFT(U)_k(t) = (1 - (1 - eta S c_k)^t) * sum_b y_bk / c_k,   c_k = number of blades covering k,
    # which tends to the coverage-weighted baseline of Section 6.
    n, s, steps = 16, 4, 7
    geom = _geom(n=n, s=s, angles=(0.0, 0.9, 1.9, 2.6), lines=(4, 5, 6, 3), shifts=np.zeros(s))
    rng = np.random.default_rng(10)
    masks = O.blade_masks(geom)
    y = masks * _crandn(rng, 4, n, n)
    cover = masks.sum(0)
    eta = 0.45 / (s * 4)
    r = O.reconstruct(geom, y, steps, tv_weight=0.0, lr=eta, optimizer="gd")
    u_hat = np.fft.fft2(r["proj"][0], norm="ortho")
    target = np.where(cover > 0, y.sum(0) / np.maximum(cover, 1), 0)
    want = (1 - (1 - eta * s * cover) ** steps) * target
    assert np.allclose(u_hat, want, atol=1e-13)
    # every bin holds 1/S of the image
    for b in range(s):
        assert np.allclose(r["vol"][0, b], r["proj"][0] / s, atol=1e-14)
    # the limit is the coverage-weighted baseline
    far = O.reconstruct(geom, y, 400, tv_weight=0.0, lr=eta, optimizer="gd")
    assert np.allclose(far["proj"][0], O.coverage_baseline(y, masks), atol=1e-10)


# ------------------------------------------------------------------ baselines and PSNR (Section 6)

def _dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) / math.sqrt(n)


@pytest.mark.parametrize("window", [1, 2, 3, 4])
def test_window_baseline_keeps_the_covered_spectrum_of_a_static_image(window):
    # every blade of a static image carries the same values where it is measured, so
    # averaging over the blades of a window returns the image's own spectrum on the union
    # of their masks and zero elsewhere (brute-force DFT matrices, not the FFT)
    n = 12
    geom = _geom(n=n, s=2, angles=(0.0, 0.6, 1.5, 2.4), lines=(3, 4, 5, 2))
    masks = O.blade_masks(geom)
    rng = np.random.default_rng(40 + window)
    x = _crandn(rng, n, n)
    f = _dft_matrix(n)
    spec = f @ x @ f.T
    y = masks * spec
    frames = O.window_baseline(y, masks, window)
    for i in range(4):
        union = masks[max(0, i - window + 1):i + 1].any(axis=0)
        want = np.conj(f).T @ (union * spec) @ np.conj(f)
        assert np.allclose(frames[i], want, atol=1e-12)


def test_window_baseline_weights_overlaps_by_coverage():
    # two blades that disagree on a shared sample average to their mean there, and a
    # sample seen by one blade only keeps that blade's value
    n = 8
    geom = _geom(n=n, s=1, angles=(0.0, 0.0), lines=(4, 2))
    masks = O.blade_masks(geom)
    rng = np.random.default_rng(44)
    y = masks * _crandn(rng, 2, n, n)
    frame = O.window_baseline(y, masks, 2)[1]
    got = _dft_matrix(n) @ frame @ _dft_matrix(n).T
    both, one = masks[0] & masks[1], masks[0] & ~masks[1]
    assert both.any() and one.any()
    assert np.allclose(got[both], 0.5 * (y[0] + y[1])[both], atol=1e-12)
    assert np.allclose(got[one], y[0][one], atol=1e-12)
    assert np.allclose(got[~masks.any(axis=0)], 0.0, atol=1e-12)


def test_window_baseline_frames_see_only_their_window():
    n, B, w = 10, 6, 3
    geom = _geom(n=n, s=1, angles=np.linspace(0.0, 2.5, B), lines=(3, 4, 5, 3, 4, 5))
    masks = O.blade_masks(geom)
    rng = np.random.default_rng(45)
    y = masks * _crandn(rng, B, n, n)
    ref = O.window_baseline(y, masks, w)
    j = 2
    y2 = y.copy()
    y2[j] += masks[j] * 0.7
    got = O.window_baseline(y2, masks, w)
    for i in range(B):
        inside = i - w + 1 <= j <= i
        assert np.array_equal(got[i], ref[i]) != inside, i
    # a window of every blade ending at the last frame is the static baseline
    assert np.allclose(O.window_baseline(y, masks, B)[-1], O.coverage_baseline(y, masks), atol=1e-14)


def test_psnr_closed_form():
    rng = np.random.default_rng(46)
    truth = _crandn(rng, 9, 11)
    c = 0.03
    image = truth * (1.0 + c / np.abs(truth))  # every magnitude off by exactly c
    peak = np.abs(truth).max()
    assert math.isclose(O.psnr(image, truth), 20.0 * math.log10(peak / c), rel_tol=1e-12)
    # the phase does not count
    assert O.psnr(1j * truth, truth) == float("inf") and O.psnr(-truth, truth) == float("inf")
    assert O.psnr(np.abs(truth) * np.exp(1j * rng.uniform(0, 6, truth.shape)), truth) > 250.0


# ------------------------------------------------------------------ data and outputs

def test_noise_free_ground_truth_has_zero_data_loss():
    case = configs.small_case(n=32, n_spec=4, n_blades=3, lines=8, sigma=0.0)
    y = O.simulate_measurements(case, dtype=np.complex128)
    geom = O.Geometry.from_dict(case.geometry())
    from synth.phantom import ground_truth_volume
    w, f = case.layers_at(0.0)
    gt = ground_truth_volume(w, f, 4)[None]
    assert O.data_loss(O.residual(gt, geom, y)) < 1e-24
    # with noise the loss at the truth is half the masked noise energy
    case2 = configs.small_case(n=32, n_spec=4, n_blades=3, lines=8, sigma=0.01)
    y2 = O.simulate_measurements(case2, dtype=np.complex128)
    masks = O.blade_masks(geom)
    want = 0.5 * np.sum(np.abs(masks * 0.01 * case2.noise) ** 2)
    assert math.isclose(O.data_loss(O.residual(gt, geom, y2)), want, rel_tol=1e-10)


def test_render_outputs():
    rng = np.random.default_rng(11)
    v = _crandn(rng, 2, 6, 5, 5)
    proj, water, fat = O.render(v)
    assert np.allclose(water + fat, proj, atol=1e-15)
    assert np.allclose(proj, v[:, 0] + v[:, 1] + v[:, 2] + v[:, 3] + v[:, 4] + v[:, 5])
    assert np.allclose(water, v[:, 0] + v[:, 1] + v[:, 2])
    _, w2, f2 = O.render(v, split_bin=1)
    assert np.allclose(w2, v[:, 0]) and np.allclose(f2, proj - v[:, 0])


# ------------------------------------------------------------------ dynamic reductions

def test_dynamic_reductions():
    rng = np.random.default_rng(12)
    base = _crandn(rng, 3, 10, 10)
    geom_s = _geom(n=10, s=3)
    geom_d = _geom(n=10, s=3, t=4, times=(0.0, 0.5, 1.0))
    # all knots equal: identical to the static model with that volume
    vd = np.stack([base] * 4)
    assert np.allclose(O.forward(vd, geom_d), O.forward(base[None], geom_s), atol=1e-13)
    # blade times on knots see exactly that knot
    assert O.knot_weights(0.0, 4) == (0, 0.0)
    assert O.knot_weights(1.0, 4) == (2, 1.0)
    k, a = O.knot_weights(0.5, 4)
    assert k == 1 and math.isclose(a, 0.5)
    v4 = _crandn(rng, 4, 3, 10, 10)
    assert np.allclose(O.volume_at(v4, 1.0), v4[3])
    assert np.allclose(O.volume_at(v4, 2.0 / 3.0), v4[2], atol=1e-15)
    # the adjoint splits a blade onto its two knots with weights (1 - a, a)
    kres = np.zeros((3, 10, 10), dtype=np.complex128)
    kres[1] = _crandn(rng, 10, 10)
    g = O.adjoint(kres, geom_d)
    gs = O.adjoint(kres, geom_s)[0]
    assert np.allclose(g[1], 0.5 * gs) and np.allclose(g[2], 0.5 * gs)
    assert np.allclose(g[0], 0) and np.allclose(g[3], 0)


# ------------------------------------------------------------------ resume

def test_resume_is_bitwise():
    case = configs.small_case(n=24, n_spec=4, n_blades=3, lines=6, n_steps=6)
    y = O.simulate_measurements(case)
    geom = O.Geometry.from_dict(case.geometry())
    full = O.reconstruct(geom, y, 6)
    half = O.reconstruct(geom, y, 3)
    rest = O.reconstruct(geom, y, 3, state=half)
    assert np.array_equal(full["vol"], rest["vol"])
    assert np.array_equal(full["history"][3:], rest["history"])


def test_cyclic_schedule_uses_one_blade_per_step():
    case = configs.small_case(n=24, n_spec=3, n_blades=3, lines=6)
    y = O.simulate_measurements(case)
    geom = O.Geometry.from_dict(case.geometry())
    r = O.reconstruct(geom, y, 1, schedule="cyclic", tv_weight=0.0, lr=0.3, optimizer="gd")
    g = O.adjoint(O.residual(np.zeros((1, 3, 24, 24)), geom, y, [0]), geom, [0])
    assert np.allclose(r["vol"], -0.3 * g, atol=1e-15)


# ------------------------------------------------------------------ schedules and data weight (Section 4.3)

def test_splitmix64_published_outputs():
    # the generator's first three outputs from state 0 (each output advances the state
    # by the golden gamma), as published with the algorithm
    g = 0x9E3779B97F4A7C15
    assert [O.splitmix64(0), O.splitmix64(g), O.splitmix64((2 * g) & ((1 << 64) - 1))] == \
        [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_random_schedule_draws_every_blade_about_equally():
    B, n = 7, 7000
    counts = np.bincount([O.random_blade(5, t, B) for t in range(n)], minlength=B)
    chi2 = float(np.sum((counts - n / B) ** 2 / (n / B)))
    assert chi2 < 30.0  # 6 degrees of freedom: p < 1e-4 beyond 30
    assert [O.random_blade(5, t, B) for t in range(20)] != [O.random_blade(6, t, B) for t in range(20)]


def test_random_schedule_steps_use_their_blade_alone():
    n = 16
    geom = _geom(n=n, s=2, angles=(0.0, 0.8, 1.7, 2.5), lines=(4, 5, 6, 3))
    rng = np.random.default_rng(50)
    y = O.blade_masks(geom) * _crandn(rng, 4, n, n)
    r = O.reconstruct(geom, y, 3, tv_weight=0.0, lr=0.1, optimizer="gd", schedule="random", seed=9)
    vol = np.zeros((1, 2, n, n), dtype=np.complex128)
    for t in range(3):
        g, _ = O.gradient(vol, geom, y, 0.0, 1e-3, 0.0, [O.random_blade(9, t, 4)])
        vol = vol - 0.1 * g
    assert np.allclose(r["vol"], vol, atol=1e-14)


def test_data_weight_scales_the_data_term_only():
    n = 12
    geom = _geom(n=n, s=3)
    rng = np.random.default_rng(51)
    vol = _crandn(rng, 1, 3, n, n)
    y = O.blade_masks(geom) * _crandn(rng, 3, n, n)
    g1, d1 = O.gradient(vol, geom, y, 0.0, 1e-3)
    g3, d3 = O.gradient(vol, geom, y, 0.0, 1e-3, data_weight=3.0)
    assert np.allclose(g3, 3.0 * g1, rtol=1e-13) and math.isclose(d3, 3.0 * d1, rel_tol=1e-13)
    tv = O.tv_grad(vol, 1e-3)
    gt, _ = O.gradient(vol, geom, y, 0.5, 1e-3, data_weight=2.0)
    assert np.allclose(gt, 2.0 * g1 + 0.5 * tv, rtol=1e-12)
