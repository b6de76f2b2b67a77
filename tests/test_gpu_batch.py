"""GPU tests of sfw_solve_batch: independent solves on several workspaces at once.

Every item of a batch must come out exactly as the same problem solved alone (the solver is
deterministic and the items share nothing), whichever workspace takes it; a failing item
fails alone and is named. Problems: the first volumes of the batched-solve workload
(synth.draw_batch), y built with the library's forward model.
"""
import os

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


VOL_MAX, PSF_MAX, MAX_ATOMS = (48, 96, 96), (33, 17, 17), 96


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
    and on new ones, give the same atoms; the repeats replay the evaluation chain from HIP
    graphs, captured by several threads at once."""
    wss, probs, data = batch
    opts = _opts(L, probs[0])
    sg = [float(np.float32(v)) for v in probs[0].config.sigma_grid]
    replay = L.default_options(mode="BSFW", sigma_grid=sg, d_grid=probs[0].config.d_grid, graphs=1)
    say("sfw_solve_batch three times: reused workspaces, then new ones (graphs)")
    first = L.sfw_solve_batch(wss, data, opts)
    again = L.sfw_solve_batch(wss, data, replay)
    streams = [torch.cuda.Stream() for _ in range(2)]
    fresh_ws = [L.Workspace(VOL_MAX, PSF_MAX, MAX_ATOMS, stream=s) for s in streams]
    try:
        fresh = L.sfw_solve_batch(fresh_ws, data, replay)
    finally:
        for w in fresh_ws:
            w.close()
    for i in range(len(data)):
        assert np.array_equal(first[i][0], again[i][0]), ("reused", i)
        assert np.array_equal(first[i][0], fresh[i][0]), ("fresh", i)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_batch_items_match_oracle(L):
    """Two items of the batched-solve workload (volumes 2 and 4 of synth.draw_batch) solved by
    sfw_solve_batch on two workspaces, on the oracle's observations, against the oracle's
    converged BSFW solutions stored by tests/golden/make_solve_golden.py: the same number of
    masses, every centre within 0.05 voxel of the oracle's, criterion within 1e-5 (relative)."""
    import json

    import oracle
    names = [n for n in ("b2", "b4") if os.path.exists(os.path.join(GOLDEN, f"solve_{n}_bsfw.json"))]
    assert names, "no stored batch solutions"
    goldens, problems = [], []
    for name in names:
        with open(os.path.join(GOLDEN, f"solve_{name}_bsfw.json")) as fh:
            g = json.load(fh)
        i = int(name[1:])
        prob = synth.draw_batch(i + 1)[i]
        psf = prob.psf.astype(np.float32).astype(np.float64)
        clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
        y = synth.make_observation(clean, prob.noise_unit, prob.config.noise_rel)
        goldens.append(g)
        problems.append((dev(y), dev(psf), g["lambda"]))
    streams = [torch.cuda.Stream() for _ in range(2)]
    wss = [L.Workspace(VOL_MAX, PSF_MAX, MAX_ATOMS, stream=s) for s in streams]
    try:
        torch.cuda.synchronize()
        say("sfw_solve_batch on stored oracle solutions", names)
        opts = L.default_options(mode="BSFW", sigma_grid=goldens[0]["sigma_grid"],
                                 d_grid=goldens[0]["d_grid"])
        res = L.sfw_solve_batch(wss, problems, opts)
    finally:
        for w in wss:
            w.close()
    for name, g, (atoms, st, code) in zip(names, goldens, res):
        ref = np.asarray(g["atoms"])
        say(name, "atoms", atoms.shape[0], "oracle", ref.shape[0], "criterion", st["criterion"],
            "oracle", g["criterion"])
        assert code == L.SFW_OK
        assert atoms.shape[0] == ref.shape[0]
        for t in ref:
            assert np.min(np.linalg.norm(atoms[:, 1:4] - t[1:4], axis=1)) <= 0.05
        assert abs(st["criterion"] - g["criterion"]) <= 1e-5 * g["criterion"]
