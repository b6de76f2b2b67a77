"""GPU parity of the autograd layer over the forward model and the criterion.

ForwardModel's backward (sfw_forward_vjp) is compared with the FP64 oracle's
vector-Jacobian product (relative L2 1e-4, the gradient bar) and, at 128x128x64 with 50
atoms, with central differences of the FP64 forward model at h = 1e-3. Criterion's
backward must be the gradient sfw_residual_grad returns, and a torch-optimizer slide over
all 6N parameters through it must descend.
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


@pytest.fixture(scope="module")
def AG(L):
    from paper_2009_05473_amd import autograd
    return autograd


@pytest.fixture(scope="module")
def ws(L):
    w = L.Workspace((64, 128, 128), (31, 15, 15), 64)
    yield w
    w.close()


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dtype))).cuda()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def say(*msg):
    print("[case]", *msg, flush=True)


def _problem(name):
    prob = config_problem(name)
    atoms = parity_atoms(prob)
    psf = f32(prob.psf)
    clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
    y = f32(synth.make_observation(clean, prob.noise_unit, prob.config.noise_rel))
    return prob, atoms, psf, y


def _cotangent(shape, seed):
    return f32(np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_forward_model_vjp_parity(L, AG, ws, name):
    prob, atoms, psf, _ = _problem(name)
    g = _cotangent(prob.shape, prob.seed + 77)
    say("ForwardModel backward", name, prob.shape, "atoms", len(atoms))
    x = dev(atoms).requires_grad_(True)
    phi = AG.forward_model(x, dev(psf), ws, prob.shape)
    phi.backward(dev(g))
    torch.cuda.synchronize()
    assert rel_l2(phi.detach().cpu().numpy(), oracle.blur(oracle.render(prob.shape, atoms), psf)) \
        <= 1e-5
    want = oracle.forward_vjp(g, atoms, psf)
    got = x.grad.cpu().numpy()
    assert rel_l2(got, want) <= 1e-4
    for c in range(6):
        assert rel_l2(got[:, c], want[:, c]) <= 2e-4, c


def test_forward_model_vjp_edge(L, AG, ws):
    """Ragged volume, PSF wider than the volume along z, one centre on a voxel, n = 0."""
    shape, psf_shape = (11, 29, 37), (15, 5, 3)
    rng = np.random.default_rng(4242)
    psf = f32(np.abs(rng.standard_normal(psf_shape)) + 0.05)
    atoms = f32(synth.random_atoms(rng, 4, shape))
    atoms[0, 1:4] = np.round(atoms[0, 1:4])
    g = _cotangent(shape, 4243)
    say("sfw_forward_vjp edge", shape, psf_shape)
    got = L.sfw_forward_vjp(ws, dev(psf), dev(g), dev(atoms))
    torch.cuda.synchronize()
    assert rel_l2(got.cpu().numpy(), oracle.forward_vjp(g, atoms, psf)) <= 1e-4
    # no atoms: only the adjoint runs, and it is left in the workspace
    assert L.sfw_forward_vjp(ws, dev(psf), dev(g), None).shape == (0, 6)


def test_forward_model_central_differences_c3(L, AG, ws):
    """h = 1e-3 central differences of <g, Phi mu> in FP64 for 8 of the 50 atoms.

    <g, H * f> = <Phi^T g, f> (the adjoint identity the oracle is pinned to), and f is a sum
    over atoms, so one parameter's difference quotient only needs that atom's profile."""
    prob, atoms, psf, _ = _problem("c3")
    g = _cotangent(prob.shape, prob.seed + 78)
    say("ForwardModel FD h=1e-3", prob.shape)
    x = dev(atoms).requires_grad_(True)
    AG.forward_model(x, dev(psf), ws, prob.shape).backward(dev(g))
    torch.cuda.synchronize()
    got = x.grad.cpu().numpy()
    q = oracle.adjoint(g, psf)
    h = 1e-3
    pick = list(range(0, 50, 7))
    fd = np.zeros((len(pick), 6))
    for i, n in enumerate(pick):
        for p in range(6):
            vals = []
            for sgn in (1.0, -1.0):
                a = atoms[n].copy()
                a[p] += sgn * h
                vals.append(a[0] * np.sum(q * oracle.atom_profile(prob.shape, *a[1:])))
            fd[i, p] = (vals[0] - vals[1]) / (2 * h)
    assert rel_l2(got[pick], fd) <= 1e-4
    for c in range(6):
        assert rel_l2(got[pick, c], fd[:, c]) <= 2e-4, c


def test_criterion_function_is_analytic_gradient(L, AG, ws):
    prob, atoms, psf, y = _problem("c3")
    lam = 1.3
    say("Criterion backward c3")
    x = dev(atoms).requires_grad_(True)
    C = AG.criterion(x, dev(y), dev(psf), lam, ws)
    C.backward()
    _, loss, grad = L.sfw_residual_grad(ws, dev(psf), dev(y), lam, dev(atoms), want_r=False)
    torch.cuda.synchronize()
    assert float(C.detach()) == float(loss.cpu()[0])
    assert np.array_equal(x.grad.cpu().numpy(), grad.cpu().numpy())
    C_o, g_o, _, _ = oracle.criterion_and_grad(y, atoms, psf, lam)
    assert rel_err(float(C.detach()), C_o) <= 1e-5
    assert rel_l2(x.grad.cpu().numpy(), g_o) <= 1e-4


def test_slide_over_all_parameters_descends(L, AG, ws):
    """torch.optim.LBFGS through Criterion from perturbed parameters at 128x128x64, 50 atoms:
    it ends well below where it started, at least as low as the truth, with the centres
    closer to the truth."""
    prob, atoms, psf, y = _problem("c3")
    lam = 1.3
    nz, ny, nx = prob.shape
    lo = [0.0, 0.0, 0.0, 0.0, synth.SIGMA_BOUNDS[0], synth.D_BOUNDS[0]]
    hi = [np.inf, nx - 1.0, ny - 1.0, nz - 1.0, synth.SIGMA_BOUNDS[1], synth.D_BOUNDS[1]]
    say("slide LBFGS c3")
    H, Y = dev(psf), dev(y)
    x0 = dev(atoms)
    c0 = float(AG.criterion(x0, Y, H, lam, ws))
    c_true = float(AG.criterion(dev(f32(prob.atoms_true)), Y, H, lam, ws))
    x, hist = AG.slide(ws, Y, H, lam, x0, lo, hi, max_iter=40)
    c1 = float(AG.criterion(x, Y, H, lam, ws))
    say("C start", c0, "truth", c_true, "end", c1, "history", [round(v, 4) for v in hist])
    assert hist[0] == pytest.approx(c0, rel=1e-12)
    assert c1 <= c_true < c0
    # the slide moves the centres toward the truth
    err0 = np.abs(atoms[:, 1:4] - prob.atoms_true[:, 1:4]).max()
    err1 = np.abs(x.cpu().numpy()[:, 1:4] - prob.atoms_true[:, 1:4]).max()
    assert err1 < err0
