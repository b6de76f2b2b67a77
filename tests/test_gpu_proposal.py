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
