"""GPU tests of sfw_solve_batch: independent solves on several workspaces at once.

Every item of a batch must come out exactly as the same problem solved alone (the solver is
deterministic and the items share nothing), whichever workspace takes it; a failing item
fails alone and is named. Problems: the first volumes of the batched-solve workload
(synth.draw_batch), y built with the library's forward model.
"""
import numpy as np
import pytest

from paper_2009_05473_amd import synth

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


VOL_MAX, PSF_MAX, MAX_ATOMS = (48, 96, 96), (29, 15, 15), 96


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def build(L, ws, prob):
    """(y, H, lambda) of one batch problem, as the benchmark builds them. ws must enqueue on
    torch's current stream, which the tensor arithmetic here uses too."""
    cfg = prob.config
    H = dev(prob.psf)
    clean = L.sfw_forward(ws, H, dev(prob.atoms_true), prob.shape)
    y = (clean + cfg.noise_rel * clean.max() * dev(prob.noise_unit)).contiguous()
    sg = [float(np.float32(v)) for v in cfg.sigma_grid]
    _, best = L.sfw_certificate(ws, H, y, 1.0, sg, cfg.d_grid)
    lam = float(np.float32(cfg.lambda_rel * best["eta"]))
    return y, H, lam


@pytest.fixture(scope="module")
def batch(L):
    streams = [torch.cuda.Stream() for _ in range(3)]
    wss = [L.Workspace(VOL_MAX, PSF_MAX, MAX_ATOMS, stream=s) for s in streams]
    probs = synth.draw_batch(6)
    with L.Workspace(VOL_MAX, PSF_MAX, MAX_ATOMS) as builder:  # torch's current stream
        data = [build(L, builder, p) for p in probs]
    torch.cuda.synchronize()  # the solving workspaces run on their own streams
    yield wss, probs, data
    for w in wss:
        w.close()


def _opts(L, prob):
    sg = [float(np.float32(v)) for v in prob.config.sigma_grid]
    return L.default_options(mode="BSFW", sigma_grid=sg, d_grid=prob.config.d_grid)


def test_batch_equals_solves_one_at_a_time(L, batch):
    wss, probs, data = batch
    opts = _opts(L, probs[0])  # the grids are the same for every batch volume
    say("sequential solves of", len(probs), "batch volumes")
    alone = [L.sfw_solve(wss[0], y, H, lam, opts) for (y, H, lam) in data]
    say("sfw_solve_batch on", len(wss), "workspaces")
    together = L.sfw_solve_batch(wss, data, opts)
    for i, ((a0, s0, c0), (a1, s1, c1)) in enumerate(zip(alone, together)):
        assert c0 == c1 == L.SFW_OK, i
        assert np.array_equal(a0, a1), i
        assert s0["criterion"] == s1["criterion"] and s0["iterations"] == s1["iterations"], i
    for (atoms, stats, _), p in zip(together, probs):
        assert stats["converged"] == 1 and len(atoms) >= 1, p.config.name


def test_batch_edge_cases(L, batch):
    wss, probs, data = batch
    opts = _opts(L, probs[0])
    say("sfw_solve_batch: no items, more workspaces than items, one workspace")
    assert L.sfw_solve_batch(wss, [], opts) == []
    one = L.sfw_solve_batch(wss, data[:1], opts)
    alone = L.sfw_solve_batch(wss[:1], data[:1], opts)
    assert np.array_equal(one[0][0], alone[0][0])


def test_batch_failing_item_is_named(L, batch):
    wss, probs, data = batch
    opts = _opts(L, probs[0])
    y_bad = data[1][0].clone()
    y_bad[3, 4, 5] = float("nan")
    torch.cuda.synchronize()
    items = [data[0], (y_bad, data[1][1], data[1][2]), data[2]]
    say("sfw_solve_batch with NaN in item 1")
    with pytest.raises(L.SfwError) as e:
        L.sfw_solve_batch(wss, items, opts)
    assert e.value.code == L.SFW_EINVAL and "batch item 1" in str(e.value)


def test_batch_repeats_exactly_on_fresh_and_reused_workspaces(L, batch):
    """The same items solved again, on workspaces that just solved them (warm LASSO caches)
    and on new ones, give the same atoms."""
    wss, probs, data = batch
    opts = _opts(L, probs[0])
    say("sfw_solve_batch three times: reused workspaces, then new ones")
    first = L.sfw_solve_batch(wss, data, opts)
    again = L.sfw_solve_batch(wss, data, opts)
    streams = [torch.cuda.Stream() for _ in range(2)]
    fresh_ws = [L.Workspace(VOL_MAX, PSF_MAX, MAX_ATOMS, stream=s) for s in streams]
    try:
        fresh = L.sfw_solve_batch(fresh_ws, data, opts)
    finally:
        for w in fresh_ws:
            w.close()
    for i in range(len(data)):
        assert np.array_equal(first[i][0], again[i][0]), ("reused", i)
        assert np.array_equal(first[i][0], fresh[i][0]), ("fresh", i)
