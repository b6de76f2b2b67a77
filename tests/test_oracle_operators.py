"""Pins of the oracle's operators (atom, render, blur, adjoint, criterion, gradient, certificate).

Each test ties an oracle function to something other than itself: a closed form,
an invariant, brute force on a tiny input, or a library routine that implements a
special case. CPU only.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2009_05473_amd import synth


def brute_conv(f, h):
    """Pure-Python (H * f)(s) = sum_t H[c+t] f(s-t), zero outside."""
    nz, ny, nx = f.shape
    pz, py, px = h.shape
    cz, cy, cx = (pz - 1) // 2, (py - 1) // 2, (px - 1) // 2
    out = np.zeros_like(f)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for kz in range(pz):
                    for ky in range(py):
                        for kx in range(px):
                            sz, sy, sx = z - (kz - cz), y - (ky - cy), x - (kx - cx)
                            if 0 <= sz < nz and 0 <= sy < ny and 0 <= sx < nx:
                                acc += h[kz, ky, kx] * f[sz, sy, sx]
                out[z, y, x] = acc
    return out


# ------------------------------------------------------------------ atom

@pytest.mark.parametrize("d", [1.3, 1.5, 2.0, 2.5, 3.0])
def test_atom_closed_form_points(d):
    shape = (9, 9, 9)
    sigma = 2.0
    g = oracle.atom_profile(shape, 4.0, 4.0, 4.0, sigma, d)
    assert g[4, 4, 4] == 1.0  # peak value 1 at the centre
    # at r = sigma the atom is exp(-1/2) for every exponent
    assert g[4, 4, 6] == pytest.approx(math.exp(-0.5), rel=1e-14)
    assert g[6, 4, 4] == pytest.approx(math.exp(-0.5), rel=1e-14)
    # at r = 2 sigma (= 4 voxels) the value is exp(-2^d / 2)
    assert g[4, 4, 8] == pytest.approx(math.exp(-(2.0 ** d) / 2.0), rel=1e-13)
    # along a diagonal, r = sqrt(3) * 2
    r = math.sqrt(12.0)
    assert g[6, 6, 6] == pytest.approx(math.exp(-((r / sigma) ** d) / 2.0), rel=1e-13)


def test_atom_d2_is_textbook_gaussian():
    from scipy.stats import multivariate_normal
    shape = (7, 8, 9)
    m = np.array([4.3, 3.7, 2.9])
    s = 1.3
    g = oracle.atom_profile(shape, *m, s, 2.0)
    z, y, x = np.meshgrid(np.arange(7), np.arange(8), np.arange(9), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pdf = multivariate_normal(mean=m, cov=s * s * np.eye(3)).pdf(pts)
    np.testing.assert_allclose(g.ravel(), pdf * (2 * math.pi * s * s) ** 1.5, rtol=1e-12, atol=1e-300)


def test_atom_radial_symmetry():
    shape = (11, 11, 11)
    g = oracle.atom_profile(shape, 5.0, 5.0, 5.0, 1.7, 1.6)
    np.testing.assert_array_equal(g, g.transpose(1, 0, 2))
    np.testing.assert_array_equal(g, g.transpose(2, 1, 0))
    np.testing.assert_array_equal(g, g[::-1, :, :])


def test_render_is_weighted_sum():
    shape = (6, 7, 8)
    atoms = np.array([[1.5, 2.0, 3.0, 1.0, 1.2, 2.0], [0.5, 5.5, 1.0, 4.0, 0.9, 1.5]])
    f = oracle.render(shape, atoms)
    want = 1.5 * oracle.atom_profile(shape, 2.0, 3.0, 1.0, 1.2, 2.0) \
        + 0.5 * oracle.atom_profile(shape, 5.5, 1.0, 4.0, 0.9, 1.5)
    np.testing.assert_allclose(f, want, rtol=1e-15)
    # peak amplitude is w at an on-grid centre (second atom far enough away)
    single = oracle.render(shape, atoms[:1])
    assert single[1, 3, 2] == 1.5


# ------------------------------------------------------------------ blur / adjoint

def test_delta_psf_gives_render():
    rng = np.random.default_rng(1)
    shape = (10, 11, 12)
    atoms = synth.random_atoms(rng, 4, shape)
    f = oracle.render(shape, atoms)
    phi = oracle.blur(f, np.ones((1, 1, 1)))
    np.testing.assert_allclose(phi, f, rtol=0, atol=1e-14)


@pytest.mark.parametrize("t", [(1, -2, 3), (0, 0, -1), (-3, 1, 0)])
def test_blur_one_hot_is_shift(t):
    """One-hot H at c + t gives (H * f)(s) = f(s - t): pins orientation and centring."""
    rng = np.random.default_rng(2)
    f = rng.standard_normal((8, 9, 10))
    h = np.zeros((7, 5, 9))
    tz, ty, tx = t
    h[3 + tz, 2 + ty, 4 + tx] = 1.0
    phi = oracle.blur(f, h)
    want = np.zeros_like(f)
    nz, ny, nx = f.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                sz, sy, sx = z - tz, y - ty, x - tx
                if 0 <= sz < nz and 0 <= sy < ny and 0 <= sx < nx:
                    want[z, y, x] = f[sz, sy, sx]
    np.testing.assert_allclose(phi, want, atol=1e-13)
    q = oracle.adjoint(f, h)
    want_adj = np.zeros_like(f)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                sz, sy, sx = z + tz, y + ty, x + tx
                if 0 <= sz < nz and 0 <= sy < ny and 0 <= sx < nx:
                    want_adj[z, y, x] = f[sz, sy, sx]
    np.testing.assert_allclose(q, want_adj, atol=1e-13)


def test_blur_brute_force_tiny():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((5, 6, 7))
    h = rng.standard_normal((3, 5, 3))
    np.testing.assert_allclose(oracle.blur(f, h), brute_conv(f, h), rtol=1e-12, atol=1e-12)
    # PSF larger than the volume on one axis
    h2 = rng.standard_normal((9, 3, 1))
    np.testing.assert_allclose(oracle.blur(f, h2), brute_conv(f, h2), rtol=1e-12, atol=1e-12)


def test_blur_and_adjoint_match_ndimage():
    rng = np.random.default_rng(4)
    f = rng.standard_normal((12, 13, 14))
    h = rng.standard_normal((5, 7, 3))
    np.testing.assert_allclose(oracle.blur(f, h), ndimage.convolve(f, h, mode="constant", cval=0.0),
                               rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(oracle.adjoint(f, h), ndimage.correlate(f, h, mode="constant", cval=0.0),
                               rtol=1e-11, atol=1e-11)


def test_adjoint_identity():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((16, 15, 14))
    r = rng.standard_normal((16, 15, 14))
    h = rng.standard_normal((9, 5, 7))
    lhs = float(np.sum(oracle.blur(f, h) * r))
    rhs = float(np.sum(f * oracle.adjoint(r, h)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 100


def test_variances_add_for_gaussian_psf():
    """d = 2 atom blurred by a unit-sum Gaussian PSF is a Gaussian with summed variances.

    Per axis the continuous result is sigma / sqrt(sigma^2 + b^2) * exp(-D^2 / 2(sigma^2 + b^2)).
    Sampling error is ~2 exp(-2 pi^2 sigma^2 b^2 / (sigma^2 + b^2)) ~ 5e-10 here.
    """
    sig = 1.5
    bxy, bz = 1.5, 2.0
    psf = synth.gaussian_psf(bxy, bz, (29, 23, 23))  # radius >= 7 b on every axis
    shape = (37, 33, 33)
    m = (16.3, 15.6, 18.2)
    f = oracle.atom_profile(shape, *m, sig, 2.0)
    phi = oracle.blur(f, psf)
    x, y, z = oracle.coords(shape)
    vxy = sig * sig + bxy * bxy
    vz = sig * sig + bz * bz
    want = (sig * sig / vxy) * (sig / math.sqrt(vz)) * np.exp(
        -((x - m[0]) ** 2 + (y - m[1]) ** 2) / (2 * vxy) - (z - m[2]) ** 2 / (2 * vz))
    err = np.max(np.abs(phi - want)) / np.max(want)
    assert err < 1e-8


# ------------------------------------------------------------------ criterion and gradient

def _small_problem(seed=7, n=3, shape=(14, 15, 16), psf_shape=(7, 5, 3)):
    rng = np.random.default_rng(seed)
    psf = np.abs(rng.standard_normal(psf_shape)) + 0.1  # asymmetric on purpose
    psf /= psf.sum()
    truth = synth.random_atoms(rng, n, shape, margin=2.0)
    y = oracle.blur(oracle.render(shape, truth), psf) + 0.05 * rng.standard_normal(shape)
    atoms = synth.random_atoms(rng, n, shape, margin=2.0)
    return y, psf, atoms


def test_criterion_definition():
    y, psf, atoms = _small_problem()
    lam = 0.3
    C, r = oracle.criterion(y, atoms, psf, lam)
    phi = ndimage.convolve(oracle.render(y.shape, atoms), psf, mode="constant")
    assert C == pytest.approx(0.5 * np.sum((y - phi) ** 2) + lam * atoms[:, 0].sum(), rel=1e-12)


def test_gradient_matches_central_differences():
    y, psf, atoms = _small_problem()
    lam = 0.3
    _, grad, _, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    h = 1e-5
    fd = np.zeros_like(atoms)
    for n in range(atoms.shape[0]):
        for p in range(6):
            a = atoms.copy(); a[n, p] += h
            cp, _ = oracle.criterion(y, a, psf, lam)
            a[n, p] -= 2 * h
            cm, _ = oracle.criterion(y, a, psf, lam)
            fd[n, p] = (cp - cm) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=2e-6, atol=1e-7 * np.abs(fd).max())


def test_forward_vjp_matches_central_differences():
    """d<g, Phi mu>/dtheta against central differences of the FP64 forward model."""
    y, psf, atoms = _small_problem(seed=11)
    g = np.random.default_rng(12).standard_normal(y.shape)
    vjp = oracle.forward_vjp(g, atoms, psf)
    h = 1e-5
    fd = np.zeros_like(atoms)
    for n in range(atoms.shape[0]):
        for p in range(6):
            a = atoms.copy(); a[n, p] += h
            lp = np.sum(g * oracle.blur(oracle.render(y.shape, a), psf))
            a[n, p] -= 2 * h
            lm = np.sum(g * oracle.blur(oracle.render(y.shape, a), psf))
            fd[n, p] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(vjp, fd, rtol=2e-6, atol=1e-7 * np.abs(fd).max())


def test_forward_vjp_of_residual_is_data_gradient():
    """With g = r = y - Phi mu, the product is minus the data-fit part of dC/dtheta."""
    y, psf, atoms = _small_problem(seed=13)
    lam = 0.25
    _, grad, r, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    vjp = oracle.forward_vjp(r, atoms, psf)
    data = grad.copy()
    data[:, 0] -= lam
    np.testing.assert_allclose(vjp, -data, rtol=1e-10, atol=1e-12 * np.abs(data).max())


def test_gradient_atom_on_voxel_centre_is_finite():
    y, psf, atoms = _small_problem()
    atoms[0, 1:4] = np.round(atoms[0, 1:4])  # centre exactly on a voxel
    _, grad, _, _ = oracle.criterion_and_grad(y, atoms, psf, 0.3)
    assert np.all(np.isfinite(grad))
    # FD of the m, sigma and d derivatives still matches there (d > 1)
    h = 1e-5
    for p in (1, 4, 5):
        a = atoms.copy(); a[0, p] += h
        cp, _ = oracle.criterion(y, a, psf, 0.3)
        a[0, p] -= 2 * h
        cm, _ = oracle.criterion(y, a, psf, 0.3)
        assert grad[0, p] == pytest.approx((cp - cm) / (2 * h), rel=1e-4, abs=1e-6)


def test_weight_gradient_is_certificate_identity():
    """dC/dw_n = lam (1 - eta(theta_n)) ties the gradient to the certificate."""
    y, psf, atoms = _small_problem(seed=8)
    lam = 0.2
    _, grad, _, q = oracle.criterion_and_grad(y, atoms, psf, lam)
    for n in range(atoms.shape[0]):
        eta, _ = oracle.eta_point(q, lam, atoms[n, 1:6])
        assert grad[n, 0] == pytest.approx(lam * (1.0 - eta), rel=1e-11, abs=1e-12)


def test_eta_gradient_matches_central_differences():
    y, psf, atoms = _small_problem(seed=9)
    lam = 0.25
    _, _, _, q = oracle.criterion_and_grad(y, atoms, psf, lam)
    theta = np.array([6.3, 7.1, 8.6, 1.4, 1.7])
    _, g = oracle.eta_point(q, lam, theta)
    h = 1e-6
    for p in range(5):
        tp = theta.copy(); tp[p] += h
        tm = theta.copy(); tm[p] -= h
        fd = (oracle.eta_point(q, lam, tp)[0] - oracle.eta_point(q, lam, tm)[0]) / (2 * h)
        assert g[p] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_eta_single_atom_closed_form():
    """mu = 0, y = w* a*: eta(theta*) = w* ||a*||^2 / lam and grad_m eta(theta*) = 0 (symmetry)."""
    shape = (21, 21, 21)
    psf = synth.gaussian_psf(1.0, 2.0, (15, 9, 9))
    theta = (10.0, 10.0, 10.0, 1.4, 1.8)
    a = oracle.blur(oracle.atom_profile(shape, *theta), psf)
    w, lam = 1.7, 0.4
    y = w * a
    q = oracle.adjoint(y, psf)
    eta, g = oracle.eta_point(q, lam, theta)
    assert eta == pytest.approx(w * np.sum(a * a) / lam, rel=1e-12)
    assert np.max(np.abs(g[:3])) < 1e-12 * abs(eta)


# ------------------------------------------------------------------ grid certificate

def test_lut_radius_is_minimal_cube():
    for s in (0.8, 1.0, 1.37, 2.5):
        for d in (1.5, 2.0, 2.5):
            R = oracle.lut_radius(s, d)
            lut = oracle.lut_kernel(s, d)
            assert lut.shape == (2 * R + 1,) * 3
            # on-axis voxel at distance R - 1 is above exp(-T), at R it is not
            assert lut[R, R, 2 * R - 1] >= math.exp(-oracle.T_TRUNC)
            assert lut[R, R, 2 * R] <= math.exp(-oracle.T_TRUNC)
            assert lut[R, R, R] == 1.0


def test_grid_certificate_brute_force():
    rng = np.random.default_rng(10)
    q = rng.standard_normal((6, 7, 8))
    sg, dg = (0.6, 0.9), (1.8, 2.6)
    lam = 0.7
    eta = oracle.grid_certificate(q, lam, sg, dg)
    nz, ny, nx = q.shape
    for i, s in enumerate(sg):
        for j, d in enumerate(dg):
            R = oracle.lut_radius(s, d)
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        acc = 0.0
                        for tz in range(-R, R + 1):
                            for ty in range(-R, R + 1):
                                for tx in range(-R, R + 1):
                                    sz, sy, sx = z + tz, y + ty, x + tx
                                    if 0 <= sz < nz and 0 <= sy < ny and 0 <= sx < nx:
                                        r = math.sqrt(tx * tx + ty * ty + tz * tz)
                                        acc += math.exp(-(r ** d) / (2 * s ** d)) * q[sz, sy, sx]
                        assert eta[i, j, z, y, x] == pytest.approx(acc / lam, rel=1e-10, abs=1e-12)


def test_grid_certificate_equals_eta_point_away_from_truncation():
    """For a narrow atom whose cube holds all of g above fp64 noise, the grid value is eta(theta)."""
    rng = np.random.default_rng(11)
    q = rng.standard_normal((16, 16, 16))
    eta = oracle.grid_certificate(q, 0.5, (0.7,), (2.0,), T=40.0)
    e, _ = oracle.eta_point(q, 0.5, (7.0, 8.0, 9.0, 0.7, 2.0))
    assert eta[0, 0, 9, 8, 7] == pytest.approx(e, rel=1e-12)


def test_grid_argmax_single_atom_on_voxel():
    shape = (24, 24, 24)
    psf = synth.gaussian_psf(1.0, 2.0, (15, 9, 9))
    truth = (11.0, 12.0, 13.0)
    y = 1.3 * oracle.blur(oracle.atom_profile(shape, *truth, 1.5, 2.0), psf)
    q = oracle.adjoint(y, psf)
    sg, dg = tuple(np.linspace(1, 2, 4)), (1.5, 2.0, 2.5)
    eta = oracle.grid_certificate(q, 1.0, sg, dg)
    for i in range(len(sg)):
        for j in range(len(dg)):
            _, (z, yy, x) = oracle.grid_argmax(eta[i, j])
            assert (x, yy, z) == (11, 12, 13)


def test_grid_argmax_ties_lowest_index():
    eta = np.zeros((2, 3, 4, 5, 6))
    eta[1, 0, 2, 3, 4] = 5.0
    eta[0, 2, 1, 1, 1] = 5.0
    eta[1, 2, 0, 0, 0] = 5.0
    v, idx = oracle.grid_argmax(eta)
    assert v == 5.0 and idx == (0, 2, 1, 1, 1)
    eta2 = -np.ones((1, 1, 2, 2, 2))
    eta2[0, 0, 1, 0, 1] = -0.5
    assert oracle.grid_argmax(eta2) == (-0.5, (0, 0, 1, 0, 1))  # max of eta, not of |eta|
