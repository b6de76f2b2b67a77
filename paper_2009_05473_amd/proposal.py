"""Training and evaluation of the learned proposal (sfw_net_*) on the library's kernels.

Step 1 of Algorithms 1 and 2 seeds the local ascent at the grid maximum of the certificate.
The proposal network predicts that seed instead from x = Phi^T r / lambda (see include/sfw.h);
the solver falls back to the grid whenever the ascent from the network's seed ends at
eta* <= 1, so the grid certificate still decides the stopping rule.

A training sample imitates what step 1 sees inside a solve: a volume holding N ~ U{n_lo..n_hi}
atoms drawn like the 128x128x64 workload's (centres at least 3 voxels apart, sigma ~ U[1, 2],
d = 2, w ~ U[1, 2]), its 9x9x15 Gaussian PSF and 1 % noise, lambda = 0.05 x the maximum of the
grid certificate of y, and a random subset of the atoms taken as already found (exact
parameters); the input is the adjoint of y minus their forward model, the targets are the
atoms not yet found. Every volume and subset is drawn from the seed given, the noise on the
GPU from a seeded torch generator. Forward models, certificates and adjoints are the
library's; so are the network's forward and backward passes and the optimizer.
"""
from __future__ import annotations

import time
from dataclasses import replace

import numpy as np

from . import synth


def init_params(rng, channels=32):
    """He-initialised network parameters (zero biases) in the library's master layout."""
    dims = [(channels, 1), (channels, channels), (channels, channels), (3, channels)]
    parts = []
    for co, ci in dims:
        parts.append(rng.standard_normal(co * ci * 27) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def _volume(rng, shape, n_atoms):
    cfg = replace(synth.CONFIGS["c3"], shape=tuple(shape), n_atoms=int(n_atoms))
    atoms = synth.draw_atoms(cfg, rng)
    return cfg, atoms


class Sampler:
    """Training samples on one workspace (the caller's torch stream)."""

    def __init__(self, L, shape, seed, n_range=(10, 80), subsets=4):
        import torch
        self.L, self.shape, self.n_range, self.subsets = L, tuple(shape), n_range, subsets
        cfg = synth.CONFIGS["c3"]
        self.psf = synth.gaussian_psf(cfg.psf_sigma_xy, cfg.psf_sigma_z, cfg.psf_shape)
        self.H = torch.from_numpy(self.psf.astype(np.float32)).cuda()
        self.ws = L.Workspace(self.shape, self.psf.shape, 128)
        self.rng = np.random.default_rng(seed)
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.sg = [float(np.float32(v)) for v in cfg.sigma_grid]
        self.dg = list(cfg.d_grid)
        self._queue = []

    def _new_volume(self):
        import torch
        L = self.L
        n = int(self.rng.integers(self.n_range[0], self.n_range[1] + 1))
        cfg, atoms = _volume(self.rng, self.shape, n)
        A = torch.from_numpy(atoms.astype(np.float32)).cuda()
        clean = L.sfw_forward(self.ws, self.H, A, self.shape)
        noise = torch.randn(self.shape, generator=self.gen, device="cuda", dtype=torch.float32)
        y = (clean + cfg.noise_rel * clean.max() * noise).contiguous()
        _, best = L.sfw_certificate(self.ws, self.H, y, 1.0, self.sg, self.dg)
        lam = float(np.float32(cfg.lambda_rel * best["eta"]))
        for _ in range(self.subsets):
            found = self.rng.random(n) < self.rng.uniform(0.0, 0.9)
            if found.all():
                found[self.rng.integers(n)] = False
            rest = atoms[~found]
            if found.any():
                r, _, _ = L.sfw_residual_grad(self.ws, self.H, y, lam,
                                              torch.from_numpy(atoms[found].astype(np.float32)).cuda())
            else:
                r = y
            q = L.sfw_adjoint(self.ws, self.H, r)
            self._queue.append((q, 1.0 / lam, rest))

    def next(self):
        if not self._queue:
            self._new_volume()
        return self._queue.pop(0)

    def close(self):
        self.ws.close()


def train(L, net, steps, shape=(64, 128, 128), seed=20000, lr=1e-3, log_every=0, log=None):
    """Adam steps of the network on fresh samples; returns the loss history (every log_every
    steps, and the last)."""
    sampler = Sampler(L, shape, seed)
    hist = []
    t0 = time.perf_counter()
    try:
        for i in range(steps):
            q, scale, rest = sampler.next()
            want = (log_every and (i % log_every == 0)) or i == steps - 1
            loss = net.train_step(q, scale, rest, lr * (0.3 if i > 0.7 * steps else 1.0),
                                  want_loss=bool(want))
            if want:
                hist.append((i, loss))
                if log is not None:
                    print(f"[proposal] step {i} loss {loss:.5f} ({time.perf_counter() - t0:.1f} s)",
                          file=log, flush=True)
    finally:
        sampler.close()
    return hist


def held_out(n_volumes, shape=(64, 128, 128), n_atoms=50, seed=5000):
    """Held-out problems (seeds seed + i, synth.draw_held_out's draws for seed 5000): the
    128x128x64 workload's distributions."""
    out = []
    for i in range(n_volumes):
        p = synth.draw_held_out(seed - 5000 + i, shape, n_atoms)
        out.append((p.config, p.atoms_true, p.noise_unit))
    return out


def compare(L, net, problems, log=None):
    """BSFW from mu = 0 on each problem with the grid proposal and with the network's; per
    problem the solve times, atom counts, worst distance of a true centre to the nearest
    estimated one, and the proposal counters. The order alternates (grid first on even problems,
    learned first on odd ones), and one untimed solve of the first problem warms the workspace's
    tables and tuned shapes first, so neither variant gains from running second."""
    import torch
    cfg0 = problems[0][0]
    psf = synth.gaussian_psf(cfg0.psf_sigma_xy, cfg0.psf_sigma_z, cfg0.psf_shape)
    H = torch.from_numpy(psf.astype(np.float32)).cuda()
    sg = [float(np.float32(v)) for v in cfg0.sigma_grid]
    rows = []
    with L.Workspace(cfg0.shape, psf.shape, 128) as ws:
        for cfg, atoms, noise in problems:
            A = torch.from_numpy(atoms.astype(np.float32)).cuda()
            clean = L.sfw_forward(ws, H, A, cfg.shape)
            y = (clean + cfg.noise_rel * clean.max() *
                 torch.from_numpy(noise.astype(np.float32)).cuda()).contiguous()
            _, best = L.sfw_certificate(ws, H, y, 1.0, sg, cfg.d_grid)
            lam = float(np.float32(cfg.lambda_rel * best["eta"]))
            row = {"atoms_true": int(atoms.shape[0])}
            order = (("grid", None), ("learned", net))
            if len(rows) % 2:
                order = order[::-1]
            if not rows:  # warm-up, untimed
                L.sfw_solve(ws, y, H, lam, L.default_options(mode="BSFW", sigma_grid=sg,
                                                            d_grid=cfg.d_grid))
            for name, prop in order:
                opts = L.default_options(mode="BSFW", sigma_grid=sg, d_grid=cfg.d_grid)
                if prop is not None:
                    opts.proposal = prop.handle.value
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                est, stats, code = L.sfw_solve(ws, y, H, lam, opts)
                dt = time.perf_counter() - t0
                err = max(float(np.min(np.linalg.norm(est[:, 1:4] - a[1:4], axis=1)))
                          for a in atoms) if len(est) else float("inf")
                row[name] = {"seconds": dt, "atoms": int(len(est)), "status": int(code),
                             "max_centre_error": err, "criterion": stats["criterion"],
                             "iterations": stats["iterations"],
                             "seconds_seed": stats["seconds_certificate"],
                             "seconds_ascent": stats["seconds_ascent"],
                             "eta_evaluations": stats["n_eval_eta"],
                             "proposals": stats["n_proposals"], "fallbacks": stats["n_fallbacks"],
                             "certificates": stats["n_certificates"]}
            rows.append(row)
            if log is not None:
                g, l_ = row["grid"], row["learned"]
                print(f"[proposal] grid {g['seconds']:.3f} s {g['atoms']} atoms err "
                      f"{g['max_centre_error']:.3f} | learned {l_['seconds']:.3f} s {l_['atoms']} "
                      f"atoms err {l_['max_centre_error']:.3f} fallbacks {l_['fallbacks']}/"
                      f"{l_['proposals']}", file=log, flush=True)
    return rows


def summarize(rows):
    g = [r["grid"] for r in rows]
    l_ = [r["learned"] for r in rows]
    return {
        "volumes": len(rows),
        "grid_seconds_mean": float(np.mean([r["seconds"] for r in g])),
        "learned_seconds_mean": float(np.mean([r["seconds"] for r in l_])),
        "speedup": float(np.sum([r["seconds"] for r in g]) / np.sum([r["seconds"] for r in l_])),
        "grid_exact_count": int(sum(r["atoms"] == row["atoms_true"] for r, row in zip(g, rows))),
        "learned_exact_count": int(sum(r["atoms"] == row["atoms_true"] for r, row in zip(l_, rows))),
        "grid_max_centre_error": float(max(r["max_centre_error"] for r in g)),
        "learned_max_centre_error": float(max(r["max_centre_error"] for r in l_)),
        "grid_seconds_seed": float(np.sum([r["seconds_seed"] for r in g])),
        "learned_seconds_seed": float(np.sum([r["seconds_seed"] for r in l_])),
        "grid_seconds_ascent": float(np.sum([r["seconds_ascent"] for r in g])),
        "learned_seconds_ascent": float(np.sum([r["seconds_ascent"] for r in l_])),
        "grid_eta_evaluations": int(sum(r["eta_evaluations"] for r in g)),
        "learned_eta_evaluations": int(sum(r["eta_evaluations"] for r in l_)),
        "proposals": int(sum(r["proposals"] for r in l_)),
        "fallbacks": int(sum(r["fallbacks"] for r in l_)),
        "grid_certificates": int(sum(r["certificates"] for r in g)),
        "learned_certificates": int(sum(r["certificates"] for r in l_)),
        "equal_counts": int(sum(a["atoms"] == b["atoms"] for a, b in zip(g, l_))),
        "per_volume": {
            "grid_seconds": [round(r["seconds"], 4) for r in g],
            "learned_seconds": [round(r["seconds"], 4) for r in l_],
            "grid_atoms": [r["atoms"] for r in g],
            "learned_atoms": [r["atoms"] for r in l_],
            "grid_max_centre_error": [round(r["max_centre_error"], 3) for r in g],
            "learned_max_centre_error": [round(r["max_centre_error"], 3) for r in l_]},
    }


def main(argv=None):
    import argparse
    import json
    import sys

    import torch
    ap = argparse.ArgumentParser(description="train the proposal network, then compare solvers")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--volumes", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=20000)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise RuntimeError("the proposal network runs on the GPU")
    from . import _lib as L
    shape = (64, 128, 128)
    with L.Net(shape) as net:
        net.set_params(init_params(np.random.default_rng(args.seed)))
        t0 = time.perf_counter()
        hist = train(L, net, args.train_steps, shape, args.seed, args.lr,
                     log_every=max(1, args.train_steps // 10), log=sys.stderr)
        t_train = time.perf_counter() - t0
        rows = compare(L, net, held_out(args.volumes, shape), log=sys.stderr)
    out = {"train_steps": args.train_steps, "train_seconds": t_train, "loss": hist,
           "summary": summarize(rows)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
