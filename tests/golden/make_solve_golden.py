"""Writes the FP64 oracle's BSFW solutions that the GPU solver's parity tests compare against.

Calls only the oracle and the seeded input drawer. Problems:
    c2      64 x 64 x 32, 10 atoms, 15 x 15 x 31 PSF, noise 0.02 max  -> solve_c2_bsfw.json
            (a few minutes on one core)
    c3      128 x 128 x 64, 50 atoms, 9 x 9 x 15 PSF, noise 0.01 max -> solve_c3_bsfw.json
    h<i>    held-out volume i of the learned-proposal comparison (same workload as c3,
            seed 5000 + i)                                          -> solve_h<i>_bsfw.json
            (each 128 x 128 x 64 solve takes hours on one core)
    b<i>    volume i of the batched-solve workload (synth.draw_batch) -> solve_b<i>_bsfw.json
Each stored solution is the oracle's BSFW result, then polished: one more sliding descent from
it with tight tolerances (gtol 1e-12, ftol 1e-16, at most 3000 iterations) and the pruning step.
SciPy's L-BFGS-B stops on its relative-decrease test once an iteration gains less than ftol |C|,
which on the 128 x 128 x 64 workload left a mass of weight 9e-5 beside one of 0.66 with
dC/dw = +1.8e-3 (its weight still wants to fall to zero); parity is judged at converged optima,
so the stored measure is the converged one. The solve's own result is kept as "atoms_solve".
Usage:
    python tests/golden/make_solve_golden.py c2 [c3 h5 h7 ...]
    python tests/golden/make_solve_golden.py --polish c3 ...   (polish a stored solve's result)
Progress (one line per BSFW iteration) goes to stderr.
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


def problem(name):
    if name in ("c2", "c3"):
        return synth.draw_problem(name)
    if name.startswith("h"):
        return synth.draw_held_out(int(name[1:]))
    if name.startswith("b"):
        i = int(name[1:])
        return synth.draw_batch(i + 1)[i]
    raise SystemExit(f"unknown problem {name!r}")


WORKLOAD = {
    "c2": "64 x 64 x 32, 10 atoms, 15 x 15 x 31 PSF, noise 0.02 max",
    "c3": "128 x 128 x 64, 50 atoms, 9 x 9 x 15 PSF, noise 0.01 max",
}


def observation(prob):
    """y as the device sees it: the FP64 forward model of the truth plus the seeded noise,
    rounded to float32; lambda by the workloads' rule, also rounded to float32."""
    cfg = prob.config
    psf = prob.psf.astype(np.float32).astype(np.float64)
    clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
    y = synth.make_observation(clean, prob.noise_unit, cfg.noise_rel)
    y = y.astype(np.float32).astype(np.float64)
    lam = float(np.float32(cfg.lambda_rel * oracle.max_grid_certificate(
        y, psf, cfg.sigma_grid, cfg.d_grid)))
    return psf, y, lam


POLISH = {"gtol": 1e-12, "ftol": 1e-16, "maxiter": 3000}


def polish(name, y, psf, lam, prob, atoms):
    """The converged optimum near the solve's result: a sliding descent with tight tolerances,
    then the pruning step (algorithm 2, steps 2b and 3b)."""
    t0 = time.time()
    C0, _ = oracle.criterion(y, atoms, psf, lam)
    out = oracle.prune(oracle.slide(y, atoms, psf, lam, prob.bounds, **POLISH))
    C1, _ = oracle.criterion(y, out, psf, lam)
    print(f"[{name}] polish: {atoms.shape[0]} -> {out.shape[0]} atoms, C {C0:.9f} -> {C1:.9f} "
          f"({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    return out, C1


def polish_stored(names):
    for name in names:
        path = os.path.join(HERE, f"solve_{name}_bsfw.json")
        with open(path) as fh:
            out = json.load(fh)
        prob = problem(name)
        psf, y, lam = observation(prob)
        assert lam == out["lambda"]
        raw = np.asarray(out.get("atoms_solve", out["atoms"]), dtype=np.float64)
        atoms, C = polish(name, y, psf, lam, prob, raw)
        out["atoms_solve"] = [[float(v) for v in a] for a in raw]
        out["criterion_solve"] = out.get("criterion_solve", out["criterion"])
        out["atoms"] = [[float(v) for v in a] for a in atoms]
        out["criterion"] = float(C)
        out["polish"] = dict(POLISH)
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(name, "atoms", len(out["atoms"]), "criterion", out["criterion"], flush=True)


def main(names):
    if names and names[0] == "--polish":
        return polish_stored(names[1:])
    for name in names:
        prob = problem(name)
        cfg = prob.config
        psf, y, lam = observation(prob)
        sg = [float(np.float32(v)) for v in cfg.sigma_grid]
        t0 = time.time()

        def log(h):
            print(f"[{name}] k {h['k']} atoms {h['n_atoms']} C {h['C']:.6f} "
                  f"eta* {h['eta_star']:.6f} ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)

        res = oracle.solve(y, psf, lam, sg, cfg.d_grid, prob.bounds, mode="BSFW", log=log)
        seconds = time.time() - t0
        atoms, C = polish(name, y, psf, lam, prob, res.atoms)
        if name.startswith("b"):
            nz, ny, nx = prob.shape
            pz, py, px = cfg.psf_shape
            wl = (f"batch volume {name[1:]}: {nx} x {ny} x {nz}, {cfg.n_atoms} atoms, "
                  f"{px} x {py} x {pz} PSF, noise 0.02 max (seed {prob.seed})")
        else:
            wl = WORKLOAD.get(name, WORKLOAD["c3"] + f", held-out volume {name[1:]} "
                              f"(seed {prob.seed})")
        out = {"workload": wl, "seed": int(prob.seed), "mode": "BSFW", "lambda": lam,
               "sigma_grid": sg, "d_grid": list(cfg.d_grid),
               "converged": bool(res.converged), "iterations": int(res.iterations),
               "largest_support": int(max([h["n_atoms"] for h in res.history] + [0])),
               "criterion": float(C), "seconds": seconds, "polish": dict(POLISH),
               "criterion_solve": float(res.criterion),
               "atoms_solve": [[float(v) for v in a] for a in res.atoms],
               "atoms": [[float(v) for v in a] for a in atoms]}
        with open(os.path.join(HERE, f"solve_{name}_bsfw.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print(name, "atoms", len(out["atoms"]), "criterion", out["criterion"],
              "seconds", round(out["seconds"]), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2"])
