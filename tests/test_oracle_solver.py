"""Pins of the oracle's LASSO, local ascent/descent, pruning and SFW/BSFW loop. CPU only."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2009_05473_amd import synth


def _columns_problem(seed, k, shape=(16, 16, 16)):
    rng = np.random.default_rng(seed)
    psf = synth.gaussian_psf(1.0, 1.5, (9, 7, 7))
    thetas = synth.random_atoms(rng, k, shape, margin=3.0)[:, 1:6]
    truth_w = rng.uniform(0.2, 1.5, size=k)
    A = oracle.lasso_columns(shape, thetas, psf)
    y = (truth_w @ A).reshape(shape) + 0.05 * rng.standard_normal(shape)
    return y, psf, thetas, A


def test_lasso_single_column_closed_form():
    y, psf, thetas, A = _columns_problem(20, 1)
    for lam in (0.01, 0.5, 1e6):
        w, G, b = oracle.lasso_weights(y, thetas, psf, lam)
        a = A[0]
        want = max(0.0, (a @ y.reshape(-1) - lam) / (a @ a))
        assert w[0] == pytest.approx(want, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("seed,k,lam", [(21, 5, 0.3), (22, 7, 2.0), (23, 4, 0.05)])
def test_lasso_kkt_and_support_enumeration(seed, k, lam):
    """The unique minimiser is the only support whose KKT system is feasible."""
    y, psf, thetas, A = _columns_problem(seed, k)
    w, G, b = oracle.lasso_weights(y, thetas, psf, lam)
    grad = G @ w - b + lam
    scale = np.abs(b).max()
    on = w > 0
    assert np.all(np.abs(grad[on]) <= 1e-9 * scale)
    assert np.all(grad[~on] >= -1e-9 * scale)
    feasible = []
    for bits in itertools.product([0, 1], repeat=k):
        S = np.array(bits, dtype=bool)
        wS = np.zeros(k)
        if S.any():
            wS[S] = np.linalg.solve(G[np.ix_(S, S)], b[S] - lam)
            if np.any(wS[S] <= 0):
                continue
        gS = G @ wS - b + lam
        if np.all(gS[~S] >= -1e-9 * scale):
            feasible.append(wS)
    assert len(feasible) == 1
    np.testing.assert_allclose(w, feasible[0], rtol=1e-8, atol=1e-12)


def test_prune_threshold():
    a = np.array([[1.0, 0, 0, 0, 1, 2], [0.0, 1, 1, 1, 1, 2], [5e-7, 2, 2, 2, 1, 2], [2e-6, 3, 3, 3, 1, 2]])
    p = oracle.prune(a)
    np.testing.assert_array_equal(p[:, 1], [0, 3])
    assert oracle.prune(np.zeros((0, 6))).shape == (0, 6)


def _c1_like(seed=1000, noise=True, n_atoms=None):
    prob = synth.draw_problem("c1", seed - 1000)
    atoms = prob.atoms_true if n_atoms is None else prob.atoms_true[:n_atoms]
    clean = oracle.blur(oracle.render(prob.shape, atoms), prob.psf)
    y = synth.make_observation(clean, prob.noise_unit, prob.config.noise_rel if noise else 0.0)
    lam = prob.config.lambda_rel * oracle.max_grid_certificate(y, prob.psf, prob.config.sigma_grid,
                                                               prob.config.d_grid)
    return prob, atoms, y, lam


def test_ascent_reaches_stationary_point():
    prob, atoms, y, lam = _c1_like()
    q = oracle.adjoint(y, prob.psf)
    eta = oracle.grid_certificate(q, lam, prob.config.sigma_grid, prob.config.d_grid)
    _, (i, j, z, yy, x) = oracle.grid_argmax(eta)
    th0 = np.array([x, yy, z, prob.config.sigma_grid[i], prob.config.d_grid[j]], float)
    th, e = oracle.ascent(q, lam, th0, y.shape, prob.bounds)
    e0, _ = oracle.eta_point(q, lam, th0)
    assert e >= e0
    _, g = oracle.eta_point(q, lam, th)
    lo = np.array([0, 0, 0, prob.bounds["sigma"][0], prob.bounds["d"][0]])
    hi = np.array([31, 31, 31, prob.bounds["sigma"][1], prob.bounds["d"][1]])
    pg = np.where((th <= lo + 1e-9) & (g < 0), 0.0, g)  # projected gradient of an ascent
    pg = np.where((th >= hi - 1e-9) & (pg > 0), 0.0, pg)
    assert np.max(np.abs(pg)) <= 1e-4 * e


def test_slide_decreases_criterion_to_stationary_point():
    prob, truth, y, lam = _c1_like()
    start = synth.perturb(truth, 1000)
    C0, _ = oracle.criterion(y, start, prob.psf, lam)
    out = oracle.slide(y, start, prob.psf, lam, prob.bounds)
    C1, g, _, _ = oracle.criterion_and_grad(y, out, prob.psf, lam)
    assert C1 < C0
    nz, ny, nx = y.shape
    lo = np.array([0.0, 0, 0, 0, prob.bounds["sigma"][0], prob.bounds["d"][0]])
    hi = np.array([np.inf, nx - 1, ny - 1, nz - 1, prob.bounds["sigma"][1], prob.bounds["d"][1]])
    pg = np.where((out <= lo + 1e-9) & (g > 0), 0.0, g)  # projected gradient of a descent
    pg = np.where((out >= hi - 1e-9) & (pg < 0), 0.0, pg)
    assert np.max(np.abs(pg)) <= 1e-4 * C1


@pytest.mark.slow
def test_bsfw_noiseless_exact_recovery_c1():
    """Tiny noiseless volume: exactly N atoms, centres within 0.05 voxel of the truth."""
    prob, truth, y, lam = _c1_like(noise=False)
    res = oracle.solve(y, prob.psf, lam, prob.config.sigma_grid, prob.config.d_grid, prob.bounds, mode="BSFW")
    assert res.converged
    assert res.atoms.shape[0] == truth.shape[0]
    for t in truth:
        dist = np.min(np.linalg.norm(res.atoms[:, 1:4] - t[1:4], axis=1))
        assert dist <= 0.05
    Cs = [h["C"] for h in res.history] + [res.criterion]
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(Cs, Cs[1:]))  # C never increases


@pytest.mark.slow
def test_sfw_and_bsfw_reach_same_criterion_c1():
    """BSFW reaches almost exactly the criterion of SFW (section 3) on a noisy c1 volume."""
    prob, truth, y, lam = _c1_like(noise=True)
    rb = oracle.solve(y, prob.psf, lam, prob.config.sigma_grid, prob.config.d_grid, prob.bounds, mode="BSFW")
    rs = oracle.solve(y, prob.psf, lam, prob.config.sigma_grid, prob.config.d_grid, prob.bounds, mode="SFW")
    assert rb.converged and rs.converged
    assert abs(rb.criterion - rs.criterion) <= 1e-3 * rs.criterion
    assert rb.atoms.shape[0] == rs.atoms.shape[0] == truth.shape[0]
    # SFW needs exactly K steps to add K atoms (plus the stopping iteration)
    assert rs.iterations == truth.shape[0] + 1


def test_merge_coincident_pins():
    """Removing zero-weighted masses and updating the measure (algorithms 1 and 2) fuses masses
    at one point of the domain: w_i delta_theta + w_j delta_theta is one mass. Pinned by what the
    measure fixes, not by the merge's own formula: (1) exact duplicates leave Phi mu unchanged
    (linearity in the weights); (2) for masses 0.03 apart the merge keeps the total weight and the
    first moment sum w theta exactly, and moves Phi mu only to second order in the separation (a
    merge that kept either mass's parameters would move it to first order); (3) masses 0.06 apart
    in any one coordinate, beyond the 0.05 tolerance, stay separate."""
    shape = (20, 20, 20)
    psf = synth.gaussian_psf(1.0, 1.5, (9, 7, 7))
    a = np.array([1.3, 9.2, 10.1, 9.7, 1.4, 2.0])
    far = np.array([0.8, 4.0, 5.0, 14.0, 1.1, 1.8])
    phi = lambda atoms: oracle.blur(oracle.render(shape, atoms), psf)
    # (1) exact duplicate
    b = a.copy()
    b[0] = 0.4
    m = oracle.merge_coincident(np.vstack([a, far, b]))
    assert m.shape == (2, 6)
    assert m[0, 0] == pytest.approx(1.7, rel=1e-15)
    ref = phi(np.vstack([a, far, b]))
    assert np.linalg.norm(phi(m) - ref) <= 1e-12 * np.linalg.norm(ref)
    # (2) 0.03 apart in every coordinate of (m, sigma, d)
    for delta in (0.03, 0.015):
        c = a + np.array([0.0, delta, -delta, delta, delta, -delta])
        c[0] = 0.6
        pair = np.vstack([a, c])
        m = oracle.merge_coincident(pair)
        assert m.shape == (1, 6)
        assert m[0, 0] == pytest.approx(a[0] + c[0], rel=1e-15)
        np.testing.assert_allclose(m[0, 0] * m[0, 1:], a[0] * a[1:] + c[0] * c[1:], rtol=1e-14)
        ref = phi(pair)
        moved = np.linalg.norm(phi(m) - ref) / np.linalg.norm(ref)
        keep_first = np.array([a[0] + c[0], *a[1:]])
        first = np.linalg.norm(phi(keep_first[None]) - ref) / np.linalg.norm(ref)
        if delta == 0.03:
            moved_03, first_03 = moved, first
    assert moved < first / 20  # second order against first order
    assert moved_03 / moved == pytest.approx(4.0, rel=0.1)  # halving delta quarters the change
    assert first_03 / first == pytest.approx(2.0, rel=0.1)
    # (3) 0.06 apart in a single coordinate: separate
    for k in range(1, 6):
        c = a.copy()
        c[k] += 0.06
        assert oracle.merge_coincident(np.vstack([a, c])).shape == (2, 6)
    # a third mass joins the first kept mass it coincides with
    c = a + np.array([0, 0.02, 0, 0, 0, 0])
    e = a + np.array([0, -0.02, 0, 0, 0, 0])
    m = oracle.merge_coincident(np.vstack([a, far, c, e]))
    assert m.shape == (2, 6) and m[0, 0] == pytest.approx(3 * a[0])
    assert m[0, 1] == pytest.approx(a[1], abs=1e-12)


def _qp_objective(G, c, w):
    return 0.5 * w @ G @ w - c @ w


def _qp_by_supports(G, c):
    """Brute force: the KKT point among all 2^k supports (positive on S, non-negative
    gradient off S); the objective's minimiser over w >= 0 for positive definite G."""
    k = c.shape[0]
    best = None
    for bits in itertools.product([0, 1], repeat=k):
        S = np.array(bits, dtype=bool)
        w = np.zeros(k)
        if S.any():
            w[S] = np.linalg.solve(G[np.ix_(S, S)], c[S])
            if np.any(w[S] <= 0):
                continue
        g = G @ w - c
        if np.all(g[~S] >= -1e-10 * np.abs(c).max()):
            assert best is None, "two KKT points of a strictly convex problem"
            best = w
    return best


def test_nnqp_diagonal_closed_form():
    d = np.array([2.0, 0.5, 4.0, 1.0, 3.0])
    c = np.array([1.0, -2.0, 3.0, 0.0, -1e-9])
    w = oracle.nnqp(np.diag(d), c)
    np.testing.assert_allclose(w, np.maximum(c, 0.0) / d, rtol=1e-12, atol=1e-15)
    assert oracle.nnqp(np.zeros((0, 0)), np.zeros(0)).shape == (0,)


@pytest.mark.parametrize("seed,k", [(31, 4), (32, 6), (33, 7)])
def test_nnqp_matches_support_enumeration(seed, k):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((2 * k + 3, k))
    G = A.T @ A
    c = rng.standard_normal(k) * 2.0
    w = oracle.nnqp(G, c)
    want = _qp_by_supports(G, c)
    np.testing.assert_allclose(w, want, rtol=1e-9, atol=1e-12)
    assert w.min() >= 0.0 and 0 < (w > 0).sum() < k  # a case with both kinds of coordinate


def test_nnqp_singular_gram_reaches_the_minimum():
    """Duplicate columns (the same atom twice) make G singular: the minimiser is not unique,
    but the objective's minimum is, and it equals the one without the duplicate."""
    rng = np.random.default_rng(34)
    A = rng.standard_normal((12, 4))
    c = rng.standard_normal(4) + 1.0
    G = A.T @ A
    A2 = np.concatenate([A, A[:, 1:2]], axis=1)
    c2 = np.append(c, c[1])
    w2 = oracle.nnqp(A2.T @ A2, c2)
    w = _qp_by_supports(G, c)
    assert _qp_objective(A2.T @ A2, c2, w2) == pytest.approx(_qp_objective(G, c, w), rel=1e-9)
    assert w2[1] + w2[4] == pytest.approx(w[1], rel=1e-6, abs=1e-9)
