"""Writes the FP64 oracle's SFW and BSFW solutions of draws of the paper's comparison (section 3,
synthetic stand-ins), which anchor the GPU runs of that comparison to the oracle.

Calls only the oracle and the seeded input drawer. One file per draw:
    python tests/golden/make_experiment_golden.py 60:4:0 80:6:2   -> experiment_60_4_0.json, ...
(n^3 voxels, N masses, repetition). Each takes minutes to tens of minutes on one core.
Each mode's stored measure is the solve's result polished to convergence (one more sliding
descent with gtol 1e-12, ftol 1e-16, then pruning; parity is judged at converged optima); the
solve's own result is kept as "atoms_solve".
    python tests/golden/make_experiment_golden.py --polish 60:4:0 ...   (polish stored files)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2009_05473_amd import synth  # noqa: E402


POLISH = {"gtol": 1e-12, "ftol": 1e-16, "maxiter": 3000}


def observation(prob):
    cfg = prob.config
    psf = prob.psf.astype(np.float32).astype(np.float64)
    clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
    y = synth.make_observation(clean, prob.noise_unit, cfg.noise_rel)
    return psf, y.astype(np.float32).astype(np.float64)  # the values the device sees


def polish(rec, y, psf, lam, prob):
    raw = np.asarray(rec.get("atoms_solve", rec["atoms"]), dtype=np.float64)
    out = oracle.prune(oracle.slide(y, raw, psf, lam, prob.bounds, **POLISH))
    C, _ = oracle.criterion(y, out, psf, lam)
    rec["atoms_solve"] = [[float(v) for v in a] for a in raw]
    rec["criterion_solve"] = rec.get("criterion_solve", rec["criterion"])
    rec["atoms"] = [[float(v) for v in a] for a in out]
    rec["criterion"] = float(C)
    rec["polish"] = dict(POLISH)


def polish_stored(specs):
    for spec in specs:
        n, N, rep = (int(v) for v in spec.split(":"))
        path = os.path.join(HERE, f"experiment_{n}_{N}_{rep}.json")
        with open(path) as fh:
            out = json.load(fh)
        prob = synth.draw_experiment(n, N, rep)
        psf, y = observation(prob)
        for mode in ("SFW", "BSFW"):
            polish(out[mode], y, psf, out["lambda"], prob)
            print(spec, mode, "atoms", len(out[mode]["atoms"]), "criterion",
                  out[mode]["criterion"], file=sys.stderr, flush=True)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)


def main(specs):
    if specs and specs[0] == "--polish":
        return polish_stored(specs[1:])
    for spec in specs:
        n, N, rep = (int(v) for v in spec.split(":"))
        prob = synth.draw_experiment(n, N, rep)
        cfg = prob.config
        psf = prob.psf.astype(np.float32).astype(np.float64)
        clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
        y = synth.make_observation(clean, prob.noise_unit, cfg.noise_rel)
        y = y.astype(np.float32).astype(np.float64)  # the values the device sees
        lam = float(np.float32(cfg.lambda_rel * oracle.max_grid_certificate(
            y, psf, cfg.sigma_grid, cfg.d_grid)))
        sg = [float(np.float32(v)) for v in cfg.sigma_grid]
        out = {"workload": f"{n}^3 voxels, {N} masses, repetition {rep} of the SFW / BSFW "
                           "comparison (32^3 workload's distributions, PSF and noise)",
               "n": n, "N": N, "rep": rep, "seed": int(prob.seed), "lambda": lam,
               "sigma_grid": sg, "d_grid": list(cfg.d_grid)}
        for mode in ("SFW", "BSFW"):
            t0 = time.time()
            res = oracle.solve(y, psf, lam, sg, cfg.d_grid, prob.bounds, mode=mode)
            out[mode] = {"converged": bool(res.converged), "iterations": int(res.iterations),
                         "largest_support": int(max([h["n_atoms"] for h in res.history] + [0])),
                         "criterion": float(res.criterion), "seconds": time.time() - t0,
                         "atoms": [[float(v) for v in a] for a in res.atoms]}
            polish(out[mode], y, psf, lam, prob)
            print(spec, mode, "atoms", len(res.atoms), "criterion", res.criterion,
                  "seconds", round(time.time() - t0), file=sys.stderr, flush=True)
        with open(os.path.join(HERE, f"experiment_{n}_{N}_{rep}.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["60:4:0", "80:6:2"])
