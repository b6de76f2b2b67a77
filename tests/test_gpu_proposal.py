"""What the trained proposal network gains over the solver without it (GPU).

The network is trained on the GPU by sfw_net_train_step (the library's forward and backward
kernels) on freshly drawn volumes, then BSFW runs from mu = 0 on held-out 128x128x64 volumes
of 50 atoms (seeds disjoint from training) with the grid maximum and with the network as step
1's seed. The grid certificate still decides (a proposal whose ascent ends at eta* <= 1
falls back to it, and the grid seeds the rest of that solve), so the learned solver must
recover the same number of atoms at the same accuracy while computing far fewer grid
certificates; the test prints the times of both, which bench.py reports at a
larger scale.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05473_amd import _lib
    return _lib


def test_trained_proposal_matches_grid_recovery(L):
    from paper_2009_05473_amd import proposal
    shape = (64, 128, 128)
    print("[case] train 1200 steps, compare on 2 held-out volumes", flush=True)
    with L.Net(shape) as net:
        net.set_params(proposal.init_params(np.random.default_rng(7)))
        hist = proposal.train(L, net, 1200, shape, seed=31000, log_every=400)
        rows = proposal.compare(L, net, proposal.held_out(2, shape, seed=6000))
    assert hist[-1][1] < 0.2 * hist[0][1]
    for r in rows:
        g, l_ = r["grid"], r["learned"]
        print("[case] grid", round(g["seconds"], 3), "s", g["atoms"], "atoms | learned",
              round(l_["seconds"], 3), "s", l_["atoms"], "atoms,", l_["fallbacks"], "of",
              l_["proposals"], "proposals fell back", flush=True)
        assert g["status"] == l_["status"] == L.SFW_OK
        assert l_["atoms"] == g["atoms"]
        assert l_["max_centre_error"] <= g["max_centre_error"] + 0.05
        # every iteration's step 1 is a proposal, a rejected proposal and a certificate, or
        # (after the one rejection) a certificate; the network spares most certificates
        assert l_["fallbacks"] <= 1
        assert l_["proposals"] + l_["certificates"] - l_["fallbacks"] == l_["iterations"]
        assert l_["certificates"] < 0.5 * g["certificates"]


def test_rejected_proposal_hands_the_solve_to_the_grid(L):
    """A network with zero weights proposes voxel 0 (a flat heatmap, ties to the lowest voxel)
    with the sigma and d of its output biases. On a noiseless volume the ascent from that
    corner stays below eta = 1, so the first proposal is rejected. From then on the grid seeds
    every iteration, and the failed ascent changes no state, so the solve must match the
    grid-only solve: the same iterations, certificates and atoms."""
    from paper_2009_05473_amd import synth
    cfg = synth.CONFIGS["c1"]
    psf = synth.gaussian_psf(cfg.psf_sigma_xy, cfg.psf_sigma_z, cfg.psf_shape)
    H = torch.from_numpy(psf.astype(np.float32)).cuda()
    atoms = synth.draw_atoms(cfg, np.random.default_rng(77))
    sg = [float(np.float32(v)) for v in cfg.sigma_grid]
    print("[case] zero-weight proposal network on the noiseless", cfg.shape, "volume", flush=True)
    with L.Workspace(cfg.shape, psf.shape, 32) as ws, L.Net(cfg.shape) as net:
        y = L.sfw_forward(ws, H, torch.from_numpy(atoms.astype(np.float32)).cuda(), cfg.shape)
        y = y.contiguous()
        _, best = L.sfw_certificate(ws, H, y, 1.0, sg, cfg.d_grid)
        lam = float(np.float32(cfg.lambda_rel * best["eta"]))
        p = np.zeros(net.num_params, dtype=np.float32)
        p[-3:] = (0.0, 1.5, 2.0)  # output-layer biases: heatmap, sigma, d
        net.set_params(p)
        runs = {}
        for name, prop in (("grid", None), ("learned", net)):
            opts = L.default_options(mode="BSFW", sigma_grid=sg, d_grid=cfg.d_grid)
            if prop is not None:
                opts.proposal = prop.handle.value
            runs[name] = L.sfw_solve(ws, y, H, lam, opts)
    (eg, sg_, cg), (el, sl, cl) = runs["grid"], runs["learned"]
    assert cg == cl == L.SFW_OK
    assert sl["n_proposals"] == 1 and sl["n_fallbacks"] == 1
    assert sg_["n_proposals"] == 0 and sg_["n_fallbacks"] == 0
    assert sl["iterations"] == sg_["iterations"]
    assert sl["n_certificates"] == sg_["n_certificates"]
    assert el.shape == eg.shape and np.allclose(el, eg, rtol=1e-6, atol=1e-6)
    assert sl["criterion"] == pytest.approx(sg_["criterion"], rel=1e-9)
