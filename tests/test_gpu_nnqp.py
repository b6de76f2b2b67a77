"""GPU parity of the batched weights QP (sfw_nnqp_batch) with the oracle's (oracle.nnqp).

Both kernels run: one wave per problem (small problems in large batches) and four.
Bars: w within 1e-9 (relative L2) of the oracle's (the problems' Gram matrices have condition
numbers up to about 1e3, so two float64 solvers agree to about 1e-13); the objective within
1e-12 (relative); the KKT conditions to 1e-9 of max |c|. The active-set path and the NNLS the
oracle calls round differently, so the bar is not bit-exactness.
"""
import numpy as np
import pytest

import oracle
from paper_2009_05473_amd import synth
from tests._common import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05473_amd import _lib
    return _lib


def say(*msg):
    print("[case]", *msg, flush=True)


def random_problem(rng, k):
    """G = A'A of a tall Gaussian A and c = A'y - lambda for y = A w_true + noise with a sparse
    non-negative w_true: a mix of positive and zero weights at the minimiser."""
    A = rng.standard_normal((2 * k + 8, k))
    w_true = rng.uniform(0.2, 1.5, size=k) * (rng.uniform(size=k) < 0.7)
    y = A @ w_true + 0.3 * rng.standard_normal(A.shape[0])
    return A.T @ A, A.T @ y - 0.5


def column_problem(rng, k, shape):
    """The weights step on the columns of k unit atoms under a Gaussian PSF (overlapping
    atoms give correlated columns)."""
    psf = synth.gaussian_psf(1.0, 1.5, (9, 7, 7))
    thetas = synth.random_atoms(rng, k, shape, margin=2.0)[:, 1:6]
    A = oracle.lasso_columns(shape, thetas, psf)
    w_true = rng.uniform(0.2, 1.5, size=k)
    y = w_true @ A + 0.05 * rng.standard_normal(A.shape[1])
    return A @ A.T, A @ y - 0.3


def pack(problems, kmax):
    n = len(problems)
    G = np.zeros((n, kmax, kmax))
    c = np.zeros((n, kmax))
    ks = np.zeros(n, dtype=np.int32)
    for p, (Gp, cp) in enumerate(problems):
        k = cp.shape[0]
        G[p, :k, :k] = Gp
        c[p, :k] = cp
        ks[p] = k
    return G, c, ks


def run(L, problems, kmax, with_k=True):
    G, c, ks = pack(problems, kmax)
    dG, dc = torch.from_numpy(G).cuda(), torch.from_numpy(c).cuda()
    dk = torch.from_numpy(ks).cuda() if with_k else None
    w, info = L.sfw_nnqp_batch(dG, dc, dk)
    torch.cuda.synchronize()
    return w.cpu().numpy(), info.cpu().numpy()


def check_kkt(G, c, w, tol=1e-9):
    scale = max(np.abs(c).max(), 1e-300)
    g = G @ w - c
    assert w.min() >= 0.0
    on = w > 0
    assert np.all(np.abs(g[on]) <= tol * scale), np.abs(g[on]).max() / scale
    assert np.all(g[~on] >= -tol * scale), g[~on].min() / scale


def objective(G, c, w):
    return 0.5 * w @ G @ w - c @ w


def test_random_batch_uneven_sizes(L):
    """One launch over 24 problems of sizes 1 to 128 (every wave-boundary size among them)."""
    rng = np.random.default_rng(4100)
    sizes = [1, 2, 3, 7, 16, 31, 32, 33, 50, 63, 64, 65, 90, 100, 127, 128, 5, 9, 17, 40, 77,
             96, 111, 128]
    problems = [random_problem(rng, k) for k in sizes]
    say("sfw_nnqp_batch random", len(sizes), "problems, kmax 128")
    w, info = run(L, problems, 128)
    for p, (G, c) in enumerate(problems):
        k = c.shape[0]
        want = oracle.nnqp(G, c)
        assert rel_l2(w[p, :k], want) <= 1e-9, (k, rel_l2(w[p, :k], want))
        assert np.all(w[p, k:] == 0.0)
        assert objective(G, c, w[p, :k]) == pytest.approx(objective(G, c, want), rel=1e-12)
        check_kkt(G, c, w[p, :k])
        assert info[p] > 0
    assert any(0 < (w[p] > 0).sum() < sizes[p] for p in range(len(sizes)))


@pytest.mark.parametrize("k,shape", [(12, (16, 16, 16)), (40, (24, 24, 24)), (91, (32, 32, 32))])
def test_gram_of_atom_columns(L, k, shape):
    rng = np.random.default_rng(4200 + k)
    G, c = column_problem(rng, k, shape)
    say("sfw_nnqp_batch atom columns", k, shape)
    w, info = run(L, [(G, c)], k, with_k=False)
    want = oracle.nnqp(G, c)
    assert rel_l2(w[0], want) <= 1e-9, rel_l2(w[0], want)
    assert objective(G, c, w[0]) == pytest.approx(objective(G, c, want), rel=1e-12)
    check_kkt(G, c, w[0])
    assert info[0] > 0


def test_all_zero_and_empty_problems(L):
    """c <= 0 gives w = 0; k = 0 gives an all-zero row; a small kmax works without k."""
    rng = np.random.default_rng(4300)
    G, _ = random_problem(rng, 6)
    neg = -np.abs(rng.standard_normal(6)) - 0.1
    say("sfw_nnqp_batch zero / empty")
    w, info = run(L, [(G, neg), (np.zeros((0, 0)), np.zeros(0)), random_problem(rng, 6)], 6)
    assert np.all(w[0] == 0.0) and np.all(w[1] == 0.0)
    assert info[1] == 0
    G2, c2 = random_problem(rng, 5)
    w2, _ = run(L, [(G2, c2)], 5, with_k=False)
    assert rel_l2(w2[0], oracle.nnqp(G2, c2)) <= 1e-9


def test_duplicated_column(L):
    """The same atom twice makes G singular (the ridge retries run): the minimum and the sum of
    the duplicated pair's weights are unique, and the KKT conditions hold."""
    rng = np.random.default_rng(4400)
    A = rng.standard_normal((30, 10))
    A = np.concatenate([A, A[:, 3:4]], axis=1)
    y = A[:, :10] @ rng.uniform(0.5, 1.5, size=10) + 0.1 * rng.standard_normal(30)
    G, c = A.T @ A, A.T @ y - 0.2
    say("sfw_nnqp_batch duplicated column")
    w, _ = run(L, [(G, c)], 11, with_k=False)
    want = oracle.nnqp(G, c)
    assert objective(G, c, w[0]) == pytest.approx(objective(G, c, want), rel=1e-9)
    assert w[0][3] + w[0][10] == pytest.approx(want[3] + want[10], rel=1e-6)
    check_kkt(G, c, w[0], tol=1e-7)


@pytest.mark.parametrize("k", [32, 50])
def test_large_batch_in_one_launch(L, k):
    """4096 problems of 32 atoms (one wave per problem) and of 50 (four waves), more workgroups
    than the chip holds at once, against the oracle on a sample."""
    rng = np.random.default_rng(4500 + k)
    base = [random_problem(rng, k) for _ in range(16)]
    problems = [base[i % 16] for i in range(4096)]
    say("sfw_nnqp_batch 4096 x", k)
    w, info = run(L, problems, k, with_k=False)
    for i in range(16):
        want = oracle.nnqp(*base[i])
        for p in (i, i + 16 * 100, i + 16 * 255):
            assert rel_l2(w[p], want) <= 1e-9
    assert np.all(info > 0)
