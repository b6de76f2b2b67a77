"""Writes the oracle's BSFW solution on the 64 x 64 x 32, 10-atom workload (noisy) to
solve_c2_bsfw.json, the reference of the GPU solver's parity test at that size.

Calls only the oracle and the seeded input drawer; takes a few minutes on one core:
    python tests/golden/make_solve_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2009_05473_amd import synth  # noqa: E402


def main():
    prob = synth.draw_problem("c2")
    cfg = prob.config
    psf = prob.psf.astype(np.float32).astype(np.float64)
    clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
    y = synth.make_observation(clean, prob.noise_unit, cfg.noise_rel)
    y = y.astype(np.float32).astype(np.float64)  # the values the device sees
    lam = float(np.float32(cfg.lambda_rel * oracle.max_grid_certificate(
        y, psf, cfg.sigma_grid, cfg.d_grid)))
    sg = [float(np.float32(v)) for v in cfg.sigma_grid]
    res = oracle.solve(y, psf, lam, sg, cfg.d_grid, prob.bounds, mode="BSFW")
    out = {"workload": "c2: 64 x 64 x 32, 10 atoms, 15 x 15 x 31 PSF, noise 0.02 max",
           "mode": "BSFW", "lambda": lam, "sigma_grid": sg, "d_grid": list(cfg.d_grid),
           "converged": bool(res.converged), "criterion": float(res.criterion),
           "atoms": [[float(v) for v in a] for a in res.atoms]}
    with open(os.path.join(HERE, "solve_c2_bsfw.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("atoms", len(out["atoms"]), "criterion", out["criterion"])


if __name__ == "__main__":
    main()
