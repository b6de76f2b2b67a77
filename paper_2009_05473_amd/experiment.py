"""The paper's comparison of SFW and BSFW (section 3) on synthetic stand-ins, on the GPU.

For each volume size n^3 and number of masses N, `reps` seeded problems (synth.draw_experiment:
the 32^3 workload's atom distributions, anisotropic Gaussian PSF and noise level stand in for
the paper's unavailable microscopy PSF and data). For each problem the library builds
y = Phi mu* + noise with its forward model, takes lambda = 0.05 x the maximum of the grid
certificate of y (the paper fixes lambda = 0.2 on an intensity scale that is not given), and
runs sfw_solve from mu = 0 in both modes with the grid proposal.

Per run it records the wall time of sfw_solve, the final criterion, the masses found, the
largest support reached and the iterations. The paper reports that BSFW reaches almost the same
criterion as SFW while running faster, and that BSFW can carry more masses than needed until
its final descent removes them; `summarize` reports exactly those quantities per (n, N):
relative criterion gap |C_BSFW - C_SFW| / C_SFW, time ratio, count agreement, and how often
BSFW's support exceeded N.

    python -m paper_2009_05473_amd.experiment --sizes 60 80 100 --counts 4 6 8 --reps 30
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import synth


def _quartiles(v):
    v = np.asarray(v, dtype=np.float64)
    return [float(np.percentile(v, 25)), float(np.median(v)), float(np.percentile(v, 75))]


def run_problem(L, ws, n, n_atoms, rep):
    """Both solves of one seeded problem; returns one record per mode."""
    import torch
    prob = synth.draw_experiment(n, n_atoms, rep)
    cfg = prob.config
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    H = dev(prob.psf)
    clean = L.sfw_forward(ws, H, dev(prob.atoms_true), prob.shape)
    Y = (clean + cfg.noise_rel * clean.max() * dev(prob.noise_unit)).contiguous()
    sg = [float(np.float32(v)) for v in cfg.sigma_grid]
    dg = [float(v) for v in cfg.d_grid]
    _, best = L.sfw_certificate(ws, H, Y, 1.0, sg, dg)
    lam = float(np.float32(cfg.lambda_rel * best["eta"]))
    out = {}
    for mode in ("SFW", "BSFW"):
        opts = L.default_options(mode=mode, sigma_grid=sg, d_grid=dg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        atoms, stats, code = L.sfw_solve(ws, Y, H, lam, opts)
        dt = time.perf_counter() - t0
        err = max(float(np.min(np.linalg.norm(atoms[:, 1:4] - t[1:4], axis=1)))
                  for t in prob.atoms_true) if len(atoms) else float("inf")
        out[mode] = {"seconds": dt, "criterion": float(stats["criterion"]),
                     "atoms": int(atoms.shape[0]), "max_support": int(stats["max_support"]),
                     "iterations": int(stats["iterations"]), "status": int(code),
                     "max_centre_error": err}
    return {"n": n, "N": n_atoms, "rep": rep, "seed": prob.seed, "lambda": lam, **out}


def summarize(records):
    """Per-(n, N) statistics of the comparison."""
    groups = {}
    for r in records:
        groups.setdefault((r["n"], r["N"]), []).append(r)
    out = []
    for (n, N), rs in sorted(groups.items()):
        gap = [abs(r["BSFW"]["criterion"] - r["SFW"]["criterion"]) / r["SFW"]["criterion"]
               for r in rs]
        ratio = [r["BSFW"]["seconds"] / r["SFW"]["seconds"] for r in rs]
        out.append({
            "n": n, "N": N, "runs": len(rs),
            "sfw_seconds_q": _quartiles([r["SFW"]["seconds"] for r in rs]),
            "bsfw_seconds_q": _quartiles([r["BSFW"]["seconds"] for r in rs]),
            "time_ratio_bsfw_over_sfw_mean": float(np.mean(ratio)),
            "criterion_gap_max": float(np.max(gap)),
            "criterion_gap_median": float(np.median(gap)),
            "counts_agree": int(sum(r["BSFW"]["atoms"] == r["SFW"]["atoms"] for r in rs)),
            "counts_equal_truth_sfw": int(sum(r["SFW"]["atoms"] == N for r in rs)),
            "counts_equal_truth_bsfw": int(sum(r["BSFW"]["atoms"] == N for r in rs)),
            "bsfw_extra_mass_runs": int(sum(r["BSFW"]["max_support"] > N for r in rs)),
            "bsfw_max_support_mean": float(np.mean([r["BSFW"]["max_support"] for r in rs])),
            "sfw_iterations_mean": float(np.mean([r["SFW"]["iterations"] for r in rs])),
            "bsfw_iterations_mean": float(np.mean([r["BSFW"]["iterations"] for r in rs])),
        })
    return out


def run(sizes, counts, reps, log=sys.stdout):
    import torch
    if not torch.cuda.is_available():  # also brings the device up before the library uses it
        raise RuntimeError("the experiment needs a GPU")
    from . import _lib as L
    nmax = max(sizes)
    psf_shape = synth.CONFIGS["c1"].psf_shape
    records = []
    with L.Workspace((nmax, nmax, nmax), psf_shape, 64) as ws:
        for n in sizes:
            for N in counts:
                t0 = time.perf_counter()
                group = [run_problem(L, ws, n, N, rep) for rep in range(reps)]
                records.extend(group)
                s = summarize(group)[0]
                s["group_seconds"] = time.perf_counter() - t0
                print(json.dumps({"group": s}), file=log, flush=True)
    return records


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sizes", type=int, nargs="+", default=[60, 80, 100])
    ap.add_argument("--counts", type=int, nargs="+", default=[4, 6, 8])
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--out", default=None, help="write every record as JSON lines here")
    args = ap.parse_args(argv)
    records = run(args.sizes, args.counts, args.reps)
    if args.out:
        with open(args.out, "w") as fh:
            for r in records:
                fh.write(json.dumps(r) + "\n")
    summary = summarize(records)
    ratio = float(np.mean([r["BSFW"]["seconds"] / r["SFW"]["seconds"] for r in records]))
    print(json.dumps({"summary": summary, "time_ratio_bsfw_over_sfw_mean": ratio,
                      "criterion_gap_max": max(s["criterion_gap_max"] for s in summary)}),
          flush=True)


if __name__ == "__main__":
    main()
