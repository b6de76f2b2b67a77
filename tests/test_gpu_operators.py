"""GPU parity of every operator of the C ABI against the FP64 oracle.

Bars (relative L2 unless stated): forward and residual 1e-5, criterion 1e-5 (relative),
adjoint and grid certificate 1e-5, gradient of C 1e-4 at perturbed (non-stationary)
parameters, eta at points 1e-5 and its gradient 1e-4, LASSO weights 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2009_05473_amd import synth
from tests._common import config_problem, parity_atoms, rel_err, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05473_amd import _lib
    return _lib


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dtype))).cuda()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def say(*msg):
    print("[case]", *msg, flush=True)


CONFIGS = ["c1", "c2", "c3"]


@pytest.fixture(params=["auto", "fft", "fft5", "mfma", "valu"])
def conv_path(request, monkeypatch):
    """Run a test on each volume convolution: the default choice (the spectral blur for large
    PSFs, else the matrix cores), the spectral blur forced (with its fused plane passes where
    they fit, and with the five separate passes), the matrix-core direct kernel and the
    LDS-tiled VALU kernel."""
    monkeypatch.delenv("SFW_BLUR_PASSES", raising=False)
    if request.param == "auto":
        monkeypatch.delenv("SFW_CONV", raising=False)
    elif request.param == "fft5":
        monkeypatch.setenv("SFW_CONV", "fft")
        monkeypatch.setenv("SFW_BLUR_PASSES", "1")
    else:
        monkeypatch.setenv("SFW_CONV", request.param)
    return request.param


@pytest.fixture(scope="module")
def ws_big(L):
    ws = L.Workspace((64, 128, 128), (31, 15, 15), 64)
    yield ws
    ws.close()


def _problem(name):
    prob = config_problem(name)
    atoms = parity_atoms(prob)
    psf = f32(prob.psf)
    clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
    y = f32(synth.make_observation(clean, prob.noise_unit, prob.config.noise_rel))
    return prob, atoms, psf, y


@pytest.mark.parametrize("name", CONFIGS)
def test_forward_parity(L, ws_big, name, conv_path):
    prob, atoms, psf, _ = _problem(name)
    say("sfw_forward", name, prob.shape, "atoms", len(atoms), conv_path)
    phi = L.sfw_forward(ws_big, dev(psf), dev(atoms), prob.shape)
    torch.cuda.synchronize()
    want = oracle.blur(oracle.render(prob.shape, atoms), psf)
    assert rel_l2(phi.cpu().numpy(), want) <= 1e-5


EDGE = [
    # (shape (nz, ny, nx), psf shape, n atoms)
    ((23, 29, 37), (7, 5, 3), 4),     # ragged in every axis
    ((8, 8, 8), (15, 9, 9), 3),       # PSF larger than the volume
    ((5, 70, 33), (1, 1, 1), 5),      # delta PSF: forward equals the render
    ((1, 1, 1), (3, 3, 3), 1),        # single voxel
    ((40, 3, 100), (9, 3, 5), 2),     # thin, several ragged x tiles
    ((17, 16, 16), (17, 1, 1), 2),    # PSF along z only, 17 taps (two z passes)
]


@pytest.mark.parametrize("shape,psf_shape,n", EDGE)
def test_forward_edge_shapes(L, ws_big, shape, psf_shape, n, conv_path):
    rng = np.random.default_rng(sum(shape) * 7 + n)
    psf = f32(np.abs(rng.standard_normal(psf_shape)) + 0.05)
    atoms = f32(synth.random_atoms(rng, n, shape))
    atoms[0, 1:4] = np.round(atoms[0, 1:4])  # one centre exactly on a voxel
    say("sfw_forward edge", shape, psf_shape, n, conv_path)
    phi = L.sfw_forward(ws_big, dev(psf), dev(atoms), shape)
    torch.cuda.synchronize()
    want = oracle.blur(oracle.render(shape, atoms), psf)
    assert rel_l2(phi.cpu().numpy(), want) <= 1e-5
    if psf_shape == (1, 1, 1):
        assert rel_l2(phi.cpu().numpy() / psf[0, 0, 0], oracle.render(shape, atoms)) <= 1e-5


def test_forward_no_atoms_is_zero(L, ws_big):
    psf = f32(synth.gaussian_psf(1.0, 2.0, (15, 9, 9)))
    say("sfw_forward n=0")
    phi = L.sfw_forward(ws_big, dev(psf), None, (9, 10, 11))
    torch.cuda.synchronize()
    assert np.all(phi.cpu().numpy() == 0.0)


@pytest.mark.parametrize("name", CONFIGS)
def test_residual_grad_parity(L, ws_big, name, conv_path):
    prob, atoms, psf, y = _problem(name)
    lam = 0.37 if name != "c3" else 1.3
    say("sfw_residual_grad", name, prob.shape, "atoms", len(atoms), conv_path)
    r, loss, grad = L.sfw_residual_grad(ws_big, dev(psf), dev(y), lam, dev(atoms))
    torch.cuda.synchronize()
    C, g, r_o, q_o = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert rel_l2(r.cpu().numpy(), r_o) <= 1e-5
    assert rel_err(loss.cpu().numpy()[0], C) <= 1e-5
    gg = grad.cpu().numpy()
    assert rel_l2(gg, g) <= 1e-4
    # every parameter block on its own scale
    for c in range(6):
        assert rel_l2(gg[:, c], g[:, c]) <= 2e-4, c


@pytest.mark.parametrize("shape", [(23, 29, 37), (23, 29, 29)])
def test_residual_grad_edge(L, ws_big, conv_path, shape):
    """Ragged sizes, on planes that are not a multiple of any tile; on the spectral paths both
    shapes run the fused plane passes (23 x 37 planes with one transform length for both axes),
    and the five separate passes where forced."""
    rng = np.random.default_rng(77)
    psf = f32(np.abs(rng.standard_normal((9, 5, 7))) + 0.05)
    psf /= psf.sum()
    truth = f32(synth.random_atoms(rng, 4, shape, margin=3))
    y = f32(oracle.blur(oracle.render(shape, truth), psf) + 0.01 * rng.standard_normal(shape))
    atoms = f32(synth.random_atoms(rng, 4, shape, margin=3))
    atoms[1, 1:4] = np.round(atoms[1, 1:4])  # centre on a voxel: finite, limit-correct gradient
    lam = 0.2
    say("sfw_residual_grad edge", shape)
    r, loss, grad = L.sfw_residual_grad(ws_big, dev(psf), dev(y), lam, dev(atoms))
    torch.cuda.synchronize()
    C, g, r_o, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert np.all(np.isfinite(grad.cpu().numpy()))
    assert rel_l2(r.cpu().numpy(), r_o) <= 1e-5
    assert rel_err(loss.cpu().numpy()[0], C) <= 1e-5
    assert rel_l2(grad.cpu().numpy(), g) <= 1e-4
    # no atoms: r = y and C = 1/2 ||y||^2
    say("sfw_residual_grad n=0")
    r0, loss0, _ = L.sfw_residual_grad(ws_big, dev(psf), dev(y), lam, None)
    torch.cuda.synchronize()
    assert np.array_equal(r0.cpu().numpy(), y.astype(np.float32))
    assert rel_err(loss0.cpu().numpy()[0], 0.5 * np.sum(y * y)) <= 1e-6


@pytest.mark.parametrize("shape,n,passes", [((40, 96, 80), 30, True), ((40, 96, 80), 30, False),
                                            ((40, 70, 70), 100, False)])
def test_residual_grad_cut_atoms(L, ws_big, shape, n, passes, monkeypatch):
    """Atoms skipped where they are exactly zero: many narrow atoms (most tiles skip most of
    them), centres outside the volume, and wide long-tailed atoms (cut radius past the whole
    volume, never skipped), against the oracle's dense sums. (40, 96, 80) runs the blur's five
    separate passes (forced) and its fused plane passes with one transform length for both
    axes; (40, 70, 70) the plane passes over ragged tiles, with more atoms than one wave's atom
    list holds (two groups of 64)."""
    if passes:
        monkeypatch.setenv("SFW_BLUR_PASSES", "1")
    else:
        monkeypatch.delenv("SFW_BLUR_PASSES", raising=False)
    rng = np.random.default_rng(2024)
    psf = f32(synth.gaussian_psf(1.0, 2.0, (15, 9, 9)))
    nz, ny, nx = shape
    atoms = np.zeros((n, 6))
    atoms[:, 0] = rng.uniform(0.5, 2.0, n)
    atoms[:, 1] = rng.uniform(-6, nx + 6, n)  # x, some outside [0, nx - 1]
    atoms[:, 2] = rng.uniform(-6, ny + 6, n)  # y
    atoms[:, 3] = rng.uniform(-4, nz + 4, n)  # z
    atoms[:, 4] = rng.uniform(0.5, 1.2, n)    # narrow
    atoms[:, 5] = rng.uniform(1.8, 3.0, n)
    atoms[:3, 4] = (3.5, 4.0, 3.8)            # wide and long-tailed
    atoms[:3, 5] = (1.2, 1.25, 1.3)
    atoms = f32(atoms)
    truth = f32(synth.random_atoms(rng, 6, shape, margin=4))
    y = f32(oracle.blur(oracle.render(shape, truth), psf) + 0.01 * rng.standard_normal(shape))
    lam = 0.3
    say("sfw_residual_grad cut atoms", shape, len(atoms))
    w = ws_big if n <= 64 else L.Workspace(shape, psf.shape, n)
    try:
        phi = L.sfw_forward(w, dev(psf), dev(atoms), shape)
        r, loss, grad = L.sfw_residual_grad(w, dev(psf), dev(y), lam, dev(atoms))
        torch.cuda.synchronize()
    finally:
        if w is not ws_big:
            w.close()
    C, g, r_o, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert rel_l2(phi.cpu().numpy(), oracle.blur(oracle.render(shape, atoms), psf)) <= 1e-5
    assert rel_l2(r.cpu().numpy(), r_o) <= 1e-5
    assert rel_err(loss.cpu().numpy()[0], C) <= 1e-5
    gg = grad.cpu().numpy()
    assert np.all(np.isfinite(gg))
    assert rel_l2(gg, g) <= 1e-4


@pytest.mark.parametrize("shape,passes", [((40, 48, 56), True), ((40, 48, 56), False),
                                          ((40, 52, 52), False)])
def test_large_psf_spectral(L, shape, passes, monkeypatch):
    """A 17 x 17 x 33 PSF (9,537 taps: more than the spectrum kernel stages in LDS, the largest
    of the batched-solve workload's 4-sigma PSFs) through the Fourier-domain blur: the five
    separate passes, the fused plane passes on 48 x 56 planes (both axes take the longer
    transform) and on 52 x 52 planes. Forward model, residual, criterion and gradient against
    the oracle."""
    monkeypatch.setenv("SFW_CONV", "fft")
    if passes:
        monkeypatch.setenv("SFW_BLUR_PASSES", "1")
    else:
        monkeypatch.delenv("SFW_BLUR_PASSES", raising=False)
    rng = np.random.default_rng(33)
    psf = f32(synth.gaussian_psf(2.0, 4.0, (33, 17, 17)))
    truth = f32(synth.random_atoms(rng, 5, shape, margin=4))
    atoms = f32(synth.random_atoms(rng, 5, shape, margin=4))
    y = f32(oracle.blur(oracle.render(shape, truth), psf) + 0.01 * rng.standard_normal(shape))
    lam = 0.25
    with L.Workspace(shape, psf.shape, 8) as w:
        say("sfw_forward / sfw_residual_grad, 17x17x33 PSF", shape)
        phi = L.sfw_forward(w, dev(psf), dev(atoms), shape)
        r, loss, grad = L.sfw_residual_grad(w, dev(psf), dev(y), lam, dev(atoms))
        torch.cuda.synchronize()
    assert rel_l2(phi.cpu().numpy(), oracle.blur(oracle.render(shape, atoms), psf)) <= 1e-5
    C, g, r_o, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert rel_l2(r.cpu().numpy(), r_o) <= 1e-5
    assert rel_err(loss.cpu().numpy()[0], C) <= 1e-5
    assert rel_l2(grad.cpu().numpy(), g) <= 1e-4


def test_residual_grad_many_atoms(L):
    """1100 atoms: more than the gradient items' kernel keeps in LDS (1024), so every item
    reads its atom again, and 18 groups of 64 in the render's atom lists; against the oracle."""
    shape = (24, 40, 48)
    n = 1100
    rng = np.random.default_rng(1100)
    psf = f32(synth.gaussian_psf(1.0, 1.5, (9, 7, 7)))
    atoms = np.zeros((n, 6))
    atoms[:, 0] = rng.uniform(0.2, 1.0, n)
    atoms[:, 1] = rng.uniform(-2, shape[2] + 2, n)
    atoms[:, 2] = rng.uniform(-2, shape[1] + 2, n)
    atoms[:, 3] = rng.uniform(-2, shape[0] + 2, n)
    atoms[:, 4] = rng.uniform(0.6, 1.6, n)
    atoms[:, 5] = rng.uniform(1.5, 2.8, n)
    atoms = f32(atoms)
    y = f32(rng.standard_normal(shape))
    lam = 0.3
    say("sfw_residual_grad", shape, "atoms", n)
    with L.Workspace(shape, psf.shape, n) as w:
        r, loss, grad = L.sfw_residual_grad(w, dev(psf), dev(y), lam, dev(atoms))
        torch.cuda.synchronize()
    C, g, r_o, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert rel_l2(r.cpu().numpy(), r_o) <= 1e-5
    assert rel_err(loss.cpu().numpy()[0], C) <= 1e-5
    assert rel_l2(grad.cpu().numpy(), g) <= 1e-4


def test_psf_spectrum_follows_h(L, ws_big, monkeypatch):
    """The spectral blur keeps the PSF spectrum between calls: overwriting H in place, and a
    PSF of another shape, must both be seen."""
    monkeypatch.setenv("SFW_CONV", "fft")
    rng = np.random.default_rng(77)
    shape = (20, 36, 30)
    atoms = f32(synth.random_atoms(rng, 5, shape))
    h1 = f32(np.abs(rng.standard_normal((9, 7, 7))) + 0.05)
    h2 = f32(np.abs(rng.standard_normal((9, 7, 7))) + 0.05)
    h3 = f32(np.abs(rng.standard_normal((5, 9, 3))) + 0.05)
    H = dev(h1)
    A = dev(atoms)
    say("PSF spectrum cache", shape)
    p1 = L.sfw_forward(ws_big, H, A, shape).cpu().numpy()
    H.copy_(dev(h2))  # same buffer, new taps
    p2 = L.sfw_forward(ws_big, H, A, shape).cpu().numpy()
    p3 = L.sfw_forward(ws_big, dev(h3), A, shape).cpu().numpy()
    p1b = L.sfw_forward(ws_big, dev(h1), A, shape).cpu().numpy()
    f = oracle.render(shape, atoms)
    assert rel_l2(p1, oracle.blur(f, h1)) <= 1e-5
    assert rel_l2(p2, oracle.blur(f, h2)) <= 1e-5
    assert rel_l2(p3, oracle.blur(f, h3)) <= 1e-5
    assert rel_l2(p1b, oracle.blur(f, h1)) <= 1e-5


def test_adjoint_parity(L, ws_big, conv_path):
    rng = np.random.default_rng(5)
    shape = (31, 45, 50)
    r = f32(rng.standard_normal(shape))
    psf = f32(rng.standard_normal((15, 9, 9)))
    say("sfw_adjoint", shape, conv_path)
    q = L.sfw_adjoint(ws_big, dev(psf), dev(r))
    torch.cuda.synchronize()
    assert rel_l2(q.cpu().numpy(), oracle.adjoint(r, psf)) <= 1e-5


def test_adjoint_identity_on_gpu(L, ws_big, conv_path):
    rng = np.random.default_rng(6)
    shape = (20, 33, 27)
    f = rng.standard_normal(shape).astype(np.float32)
    r = rng.standard_normal(shape).astype(np.float32)
    psf = rng.standard_normal((9, 7, 5)).astype(np.float32)
    say("adjoint identity", shape)
    # correlation with flip(H) is the convolution with H, so both sides use sfw_adjoint
    Hf = L.sfw_adjoint(ws_big, dev(np.ascontiguousarray(psf[::-1, ::-1, ::-1])), dev(f))
    q = L.sfw_adjoint(ws_big, dev(psf), dev(r))
    torch.cuda.synchronize()
    lhs = float(np.sum(Hf.cpu().numpy().astype(np.float64) * r))
    rhs = float(np.sum(f.astype(np.float64) * q.cpu().numpy()))
    np.testing.assert_allclose(Hf.cpu().numpy(), oracle.blur(f, psf), rtol=0,
                               atol=1e-5 * np.abs(psf).sum() * np.abs(f).max())
    assert abs(lhs - rhs) <= 1e-5 * (np.linalg.norm(f) * np.linalg.norm(r) * np.abs(psf).sum())


@pytest.fixture(params=["fft", "fft_generic", "direct"])
def cert_path(request, monkeypatch):
    """Run a test on the Fourier-domain certificate (default: fixed-length passes where the
    transform lengths allow), on its runtime-length passes only, and on the direct one."""
    monkeypatch.delenv("SFW_CERT", raising=False)
    monkeypatch.delenv("SFW_FFT", raising=False)
    if request.param == "direct":
        monkeypatch.setenv("SFW_CERT", "direct")
    elif request.param == "fft_generic":
        monkeypatch.setenv("SFW_FFT", "generic")
    return request.param


@pytest.mark.parametrize("fft", ["fixed", "generic"])
def test_profile_times_the_certificate_z_pass(L, fft, monkeypatch):
    """The cert_zinv class is timed by the z pass kernel's own start and stop events on the
    fixed-length path (128 x 128 x 64: lengths 150 x 150 x 81) and by an event pair around the
    launch on the runtime-length path: one launch per certificate either way, a positive time,
    and the same maximum."""
    monkeypatch.delenv("SFW_CERT", raising=False)
    if fft == "generic":
        monkeypatch.setenv("SFW_FFT", "generic")
    else:
        monkeypatch.delenv("SFW_FFT", raising=False)
    prob, atoms, psf, y = _problem("c3")
    sg = [float(np.float32(v)) for v in prob.config.sigma_grid]
    dg = list(prob.config.d_grid)
    say("profiled certificate", fft)
    with L.Workspace(prob.shape, psf.shape, 8) as w:
        Hd, Yd = dev(psf), dev(y)
        _, best0 = L.sfw_certificate(w, Hd, Yd, 0.9, sg, dg)
        torch.cuda.synchronize()
        L.sfw_profile_begin(w, ["cert_zinv", "cert_fft"])
        for _ in range(3):
            _, best = L.sfw_certificate(w, Hd, Yd, 0.9, sg, dg)
        torch.cuda.synchronize()
        prof = L.sfw_profile_end(w)
    n, ms = prof["cert_zinv"]
    assert n == 3 and 0.0 < ms / n < 10.0
    assert prof["cert_fft"][0] == 6  # the forward transform and the inverse y, x passes
    assert best == best0


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_certificate_parity(L, ws_big, name, cert_path):
    prob, atoms, psf, y = _problem(name)
    lam = 0.9
    sg, dg = prob.config.sigma_grid, prob.config.d_grid
    sgf = [float(np.float32(v)) for v in sg]
    say("sfw_certificate", name, prob.shape, cert_path)
    eta, best = L.sfw_certificate(ws_big, dev(psf), dev(y), lam, sgf, dg, want_eta=True)
    torch.cuda.synchronize()
    q = oracle.adjoint(y, psf)
    eta_o = oracle.grid_certificate(q, lam, sgf, dg)
    e = eta.cpu().numpy()
    assert rel_l2(e, eta_o) <= 1e-5
    v_o, idx_o = oracle.grid_argmax(eta_o)
    assert rel_err(best["eta"], v_o) <= 1e-5
    idx = (best["i_sigma"], best["i_d"], best["z"], best["y"], best["x"])
    if idx != idx_o:  # allowed only if the oracle cannot separate the two within the bar
        assert rel_err(eta_o[idx], v_o) <= 1e-5
    # the reported maximum is the maximum of the returned grid
    assert best["eta"] == e.max()
    assert best["eta"] == e[idx]


@pytest.mark.parametrize("shape,sg,dg", [
    ((6, 7, 8), (0.6, 0.9), (1.8, 2.6)),        # tiny volume, tiny kernels
    ((5, 9, 4), (2.0, 3.0), (1.5,)),             # kernels wider than the volume
    ((37, 23, 41), (1.2, 2.2, 3.1), (1.3, 2.0)), # ragged, odd grid count (one unpaired kernel)
])
def test_certificate_edge_shapes(L, ws_big, cert_path, shape, sg, dg):
    rng = np.random.default_rng(sum(shape))
    r = f32(rng.standard_normal(shape))
    psf = f32(np.abs(rng.standard_normal((5, 3, 3))) + 0.1)
    lam = 0.7
    say("sfw_certificate edge", shape, sg, dg, cert_path)
    eta, best = L.sfw_certificate(ws_big, dev(psf), dev(r), lam, list(sg), list(dg), want_eta=True)
    torch.cuda.synchronize()
    eta_o = oracle.grid_certificate(oracle.adjoint(r, psf), lam, sg, dg)
    assert rel_l2(eta.cpu().numpy(), eta_o) <= 1e-5
    v_o, idx_o = oracle.grid_argmax(eta_o)
    assert rel_err(best["eta"], v_o) <= 1e-5
    idx = (best["i_sigma"], best["i_d"], best["z"], best["y"], best["x"])
    if idx != idx_o:
        assert rel_err(eta_o[idx], v_o) <= 1e-5


@pytest.mark.parametrize("shape", [(3, 5, 250), (250, 4, 6)])
def test_certificate_long_axis(L, cert_path, shape):
    """Transform lengths past the fixed-length sizes (generic passes on that axis)."""
    rng = np.random.default_rng(shape[0])
    r = f32(rng.standard_normal(shape))
    psf = f32(np.abs(rng.standard_normal((5, 3, 3))) + 0.1)
    sg, dg = (1.0, 1.7), (2.0, 1.6)
    ws = L.Workspace(shape, psf.shape, 4)
    try:
        say("sfw_certificate long axis", shape, cert_path)
        eta, best = L.sfw_certificate(ws, dev(psf), dev(r), 0.6, list(sg), list(dg),
                                      want_eta=True)
        torch.cuda.synchronize()
        eta_o = oracle.grid_certificate(oracle.adjoint(r, psf), 0.6, sg, dg)
        assert rel_l2(eta.cpu().numpy(), eta_o) <= 1e-5
        v_o, _ = oracle.grid_argmax(eta_o)
        assert rel_err(best["eta"], v_o) <= 1e-5
    finally:
        ws.close()


def test_certificate_argmax_only_matches_grid(L, ws_big, cert_path):
    prob, atoms, psf, y = _problem("c1")
    say("sfw_certificate argmax only")
    _, b1 = L.sfw_certificate(ws_big, dev(psf), dev(y), 0.5, [1.0, 1.5], [2.0], want_eta=False)
    eta, b2 = L.sfw_certificate(ws_big, dev(psf), dev(y), 0.5, [1.0, 1.5], [2.0], want_eta=True)
    torch.cuda.synchronize()
    assert b1 == b2


@pytest.mark.parametrize("name,npts", [("c1", 1), ("c1", 6), ("c1", 8), ("c1", 11),
                                       ("c3", 1), ("c3", 8), ("c3", 11)])
def test_eta_points_parity(L, ws_big, name, npts):
    """Up to 8 points take the one-launch path (atoms as kernel arguments, 16 or 32 planes deep
    tiles, sums reduced by the last block into host memory); more take the staged path. At
    128 x 128 x 64 the points sit within 3 voxels of true atoms anywhere in the volume (where
    eta is well above the noise)."""
    prob, atoms, psf, y = _problem(name)
    lam = 0.8
    r = f32(y - oracle.blur(oracle.render(prob.shape, atoms[:1]), psf))
    q = f32(oracle.adjoint(r, psf))
    rng = np.random.default_rng(9 + npts)
    th = np.zeros((npts, 5))
    nz, ny, nx = prob.shape
    if name == "c1":
        th[:, 0:3] = rng.uniform(3, 28, size=(npts, 3))
    else:
        near = prob.atoms_true[rng.choice(len(prob.atoms_true), npts, replace=False), 1:4]
        th[:, 0:3] = np.clip(near + rng.uniform(-3, 3, size=(npts, 3)), 0,
                             np.array([nx, ny, nz]) - 1)
    th[:, 3] = rng.uniform(0.7, 3.0, size=npts)
    th[:, 4] = rng.uniform(1.3, 2.9, size=npts)
    th[0, 0:3] = np.round(th[0, 0:3])  # on a voxel centre
    th = f32(th)
    say("sfw_eta_points", th.shape)
    eta, grad = L.sfw_eta_points(ws_big, prob.shape, dev(q), lam, th)
    for i in range(th.shape[0]):
        e_o, g_o = oracle.eta_point(q, lam, th[i])
        assert rel_err(eta[i], e_o) <= 1e-5
        assert rel_l2(grad[i], g_o) <= 1e-4


def test_lasso_parity(L, ws_big):
    prob, _, psf, y = _problem("c1")
    thetas = f32(prob.atoms_true[:, 1:6])
    atoms = np.hstack([np.zeros((len(thetas), 1)), thetas])
    lam = 0.05 * oracle.max_grid_certificate(y, psf, prob.config.sigma_grid, prob.config.d_grid)
    lam = float(np.float32(lam))
    say("sfw_lasso_weights c1", len(atoms))
    w = L.sfw_lasso_weights(ws_big, dev(psf), dev(y), lam, dev(atoms)).cpu().numpy()
    w_o, G, b = oracle.lasso_weights(y, thetas, psf, lam)
    assert rel_l2(w, w_o) <= 1e-4
    grad = G @ w - b + lam
    assert np.all(np.abs(grad[w > 0]) <= 1e-4 * np.abs(b).max())
    assert np.all(grad[w == 0] >= -1e-4 * np.abs(b).max())


def test_lasso_incremental_full_size(L, ws_big):
    """BSFW's weight step at 128 x 128 x 64 with 50 atoms: the 49-atom support first, then the
    same support plus one atom (cached columns, one new Gram row summed over the new column's
    support box) against the oracle's LASSO on the 50 atoms."""
    prob, _, psf, y = _problem("c3")
    thetas = f32(prob.atoms_true[:, 1:6])
    atoms = np.hstack([np.zeros((len(thetas), 1)), thetas])
    lam = 0.05 * oracle.max_grid_certificate(y, psf, prob.config.sigma_grid, prob.config.d_grid)
    lam = float(np.float32(lam))
    Hd, Yd = dev(psf), dev(y)
    say("sfw_lasso_weights c3 49 then 50 atoms")
    L.sfw_lasso_weights(ws_big, Hd, Yd, lam, dev(atoms[:-1]))
    w = L.sfw_lasso_weights(ws_big, Hd, Yd, lam, dev(atoms)).cpu().numpy()
    w_o, G, b = oracle.lasso_weights(y, thetas, psf, lam)
    assert rel_l2(w, w_o) <= 1e-4
    grad = G @ w - b + lam
    assert np.all(np.abs(grad[w > 0]) <= 1e-4 * np.abs(b).max())
    assert np.all(grad[w == 0] >= -1e-4 * np.abs(b).max())


def test_lasso_zero_weight_case(L, ws_big):
    """A far-off atom with no signal gets weight 0 (KKT lower bound active)."""
    prob, _, psf, y = _problem("c1")
    thetas = f32(np.vstack([prob.atoms_true[:, 1:6], [[1.0, 1.0, 30.0, 1.2, 2.0]]]))
    atoms = np.hstack([np.zeros((len(thetas), 1)), thetas])
    lam = 3.0
    say("sfw_lasso_weights zero weight")
    w = L.sfw_lasso_weights(ws_big, dev(psf), dev(y), lam, dev(atoms)).cpu().numpy()
    w_o, _, _ = oracle.lasso_weights(y, thetas, psf, lam)
    assert w_o[-1] == 0.0 and w[-1] == 0.0
    assert rel_l2(w, w_o) <= 1e-4


def test_lasso_cache_follows_y_and_h_in_place(L, ws_big):
    """Cached LASSO columns and Gram rows are keyed by fingerprints of y and H: overwriting
    either in place (same pointers) gives the weights of the new data."""
    prob, _, psf, y = _problem("c1")
    thetas = f32(prob.atoms_true[:, 1:6])
    atoms = dev(np.hstack([np.zeros((len(thetas), 1)), thetas]))
    lam = 0.5
    Hd, Yd = dev(psf), dev(y)
    say("sfw_lasso_weights cache: y and H overwritten in place")
    w0 = L.sfw_lasso_weights(ws_big, Hd, Yd, lam, atoms).cpu().numpy()
    assert rel_l2(w0, oracle.lasso_weights(y, thetas, psf, lam)[0]) <= 1e-4
    y2 = f32(1.7 * y)
    Yd.copy_(dev(y2))
    w1 = L.sfw_lasso_weights(ws_big, Hd, Yd, lam, atoms).cpu().numpy()
    assert rel_l2(w1, oracle.lasso_weights(y2, thetas, psf, lam)[0]) <= 1e-4
    psf2 = f32(0.8 * psf)
    Hd.copy_(dev(psf2))
    w2 = L.sfw_lasso_weights(ws_big, Hd, Yd, lam, atoms).cpu().numpy()
    assert rel_l2(w2, oracle.lasso_weights(y2, thetas, psf2, lam)[0]) <= 1e-4
    assert rel_l2(w1, w0) > 0.1 and rel_l2(w2, w1) > 0.1


def test_lasso_reused_slots_ignore_stale_values(L):
    """Four column slots for supports that keep replacing atoms: a reused slot keeps the old
    column's values outside the new column's box, which the Gram rows must not read (boxed
    columns at 64 x 64 x 32)."""
    shape, psf_shape = (32, 64, 64), (9, 5, 5)
    rng = np.random.default_rng(4404)
    psf = np.abs(rng.standard_normal(psf_shape)) + 0.1
    psf = f32(psf / psf.sum())
    cen = np.array([[14, 14, 10], [48, 20, 16], [20, 50, 20], [50, 50, 12], [32, 32, 16],
                    [10, 40, 22], [40, 8, 9]], dtype=np.float64)
    thetas = f32(np.hstack([cen + rng.uniform(-0.4, 0.4, cen.shape),
                            rng.uniform(1.0, 1.5, (len(cen), 1)), np.full((len(cen), 1), 2.0)]))
    truth = np.hstack([rng.uniform(0.5, 2.0, (len(cen), 1)), thetas])
    y = f32(oracle.blur(oracle.render(shape, truth), psf) + 0.01 * rng.standard_normal(shape))
    lam = 0.05
    Hd, Yd = dev(psf), dev(y)
    with L.Workspace(shape, psf_shape, 4) as w:
        for sup in ([0, 1, 2], [0, 3, 4], [5, 3, 1, 6], [2, 4, 0], [6, 5]):
            say("sfw_lasso_weights reused slots", sup)
            th = thetas[sup]
            atoms = dev(np.hstack([np.zeros((len(sup), 1)), th]))
            got = L.sfw_lasso_weights(w, Hd, Yd, lam, atoms).cpu().numpy()
            assert rel_l2(got, oracle.lasso_weights(y, th, psf, lam)[0]) <= 1e-4, sup


def test_lasso_support_longer_than_inline_slot_list(L):
    """130 atoms: the Gram-row kernels take the first 128 slots from their arguments and the
    rest from the device slot list. Lattice centres 5 voxels apart keep G well conditioned."""
    shape, psf_shape = (40, 40, 40), (5, 3, 3)
    rng = np.random.default_rng(7130)
    psf = np.abs(rng.standard_normal(psf_shape)) + 0.1
    psf = f32(psf / psf.sum())
    sites = np.array([(x, y, z) for z in range(4, 36, 5) for y in range(4, 36, 5)
                      for x in range(4, 36, 5)], dtype=np.float64)
    pick = sites[rng.choice(len(sites), 130, replace=False)]
    thetas = f32(np.hstack([pick + rng.uniform(-0.4, 0.4, pick.shape),
                            rng.uniform(1.0, 1.4, (130, 1)), np.full((130, 1), 2.0)]))
    truth = np.hstack([rng.uniform(0.5, 2.0, (130, 1)), thetas])
    y = f32(oracle.blur(oracle.render(shape, truth), psf)
            + 0.01 * rng.standard_normal(shape))
    lam = 0.05
    atoms = np.hstack([np.zeros((130, 1)), thetas])
    w_o, G, b = oracle.lasso_weights(y, thetas, psf, lam)
    assert np.count_nonzero(w_o) > 120
    say("sfw_lasso_weights 130 atoms", shape, psf_shape)
    with L.Workspace(shape, psf_shape, 160) as w:
        got = L.sfw_lasso_weights(w, dev(psf), dev(y), lam, dev(atoms)).cpu().numpy()
    assert rel_l2(got, w_o) <= 1e-4
    grad = G @ got - b + lam
    assert np.all(np.abs(grad[got > 0]) <= 1e-4 * np.abs(b).max())


@pytest.mark.parametrize("psf_shape", [(9, 9, 9), (33, 21, 21)])
def test_lasso_column_psf_in_lds_or_not(L, psf_shape):
    """The LASSO column kernel stages the PSF in LDS beside its tile where both fit (9 x 9 x 9)
    and reads it by scalar loads where they do not (21 x 21 x 33: 124 KB of tile, 188 KB with
    the PSF); both against the oracle's weights."""
    shape = (40, 48, 48)
    rng = np.random.default_rng(7200 + psf_shape[0])
    psf = f32(synth.gaussian_psf(1.5, 3.0, psf_shape))
    centres = np.array([[12, 12, 10], [34, 14, 28], [14, 35, 20], [33, 33, 12], [24, 24, 30],
                        [8, 26, 22]], dtype=np.float64)
    k = len(centres)
    thetas = f32(np.hstack([centres + rng.uniform(-0.4, 0.4, centres.shape),
                            rng.uniform(1.1, 1.6, (k, 1)), rng.uniform(1.6, 2.4, (k, 1))]))
    truth = np.hstack([rng.uniform(0.5, 2.0, (k, 1)), thetas])
    y = f32(oracle.blur(oracle.render(shape, truth), psf) + 0.01 * rng.standard_normal(shape))
    lam = 0.02
    atoms = np.hstack([np.zeros((k, 1)), thetas])
    w_o, G, b = oracle.lasso_weights(y, thetas, psf, lam)
    say("sfw_lasso_weights PSF", psf_shape)
    with L.Workspace(shape, psf_shape, 8) as w:
        got = L.sfw_lasso_weights(w, dev(psf), dev(y), lam, dev(atoms)).cpu().numpy()
    assert rel_l2(got, w_o) <= 1e-4
    grad = G @ got - b + lam
    assert np.all(np.abs(grad[got > 0]) <= 1e-4 * np.abs(b).max())


def test_reductions_are_deterministic(L, ws_big):
    prob, atoms, psf, y = _problem("c3")
    say("determinism c3")
    out = []
    for _ in range(2):
        r, loss, grad = L.sfw_residual_grad(ws_big, dev(psf), dev(y), 1.0, dev(atoms))
        _, best = L.sfw_certificate(ws_big, dev(psf), r, 1.0, [1.0, 2.0], [2.0])
        torch.cuda.synchronize()
        out.append((loss.cpu().numpy().tobytes(), grad.cpu().numpy().tobytes(), best))
    assert out[0] == out[1]


def test_certificate_allocates_nothing(L):
    """The workspace reserves the certificate's arrays at creation: a later certificate on a
    larger grid (16 kernels up to radius 40) leaves the device's free memory unchanged, and a
    grid beyond the reservation is rejected (SFW_EINVAL) instead of allocating."""
    shape = (48, 40, 56)
    rng = np.random.default_rng(11)
    r = dev(rng.standard_normal(shape))
    psf = dev(np.full((3, 3, 3), 1.0 / 27))
    with L.Workspace(shape, (3, 3, 3), 8) as ws:
        say("sfw_certificate warm-up grid")
        L.sfw_certificate(ws, psf, r, 0.5, [1.0, 2.0], [2.0])
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        say("sfw_certificate 16-kernel grid, radius up to 40")
        sg = [1.0, 2.0, 3.0, 4.8]
        dg = [1.5, 2.0, 2.5, 3.0]
        _, best = L.sfw_certificate(ws, psf, r, 0.5, sg, dg)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert 0 <= best["i_sigma"] < 4 and 0 <= best["i_d"] < 4
        with pytest.raises(L.SfwError) as e:  # 17 kernels
            L.sfw_certificate(ws, psf, r, 0.5, [1.0] * 17, [2.0])
        assert e.value.code == L.SFW_EINVAL
        with pytest.raises(L.SfwError) as e:  # radius ceil(4.9 * 24^(1/1.5)) = 41
            L.sfw_certificate(ws, psf, r, 0.5, [4.9], [1.5])
        assert e.value.code == L.SFW_EINVAL and "RADIUS" in L.last_error()
