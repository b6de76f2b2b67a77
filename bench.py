#!/usr/bin/env python3
"""Throughput of the BSFW hot path on one MI355X, against its roofline and the CPU oracle.

Workload: one 128 x 128 x 64 float32 volume with 50 atoms (centres uniform in the interior
with spacing >= 3 voxels, sigma ~ U[1, 2], d = 2, w ~ U[1, 2]), anisotropic Gaussian PSF
(sigma_xy = 1, sigma_z = 2, 9 x 9 x 15 taps), Gaussian noise of 0.01 * max(Phi mu*),
lambda = 0.05 * max of the grid certificate of y, candidate grid = voxel centres x
linspace(1, 2, 4) sigmas x {1.5, 2, 2.5} exponents. The 50 evaluated atoms are the truth
perturbed (centres +-0.5, sigma x[0.9, 1.1], d +-0.1, w x[0.8, 1.2]).

One step is one pass over every row of the hot path, as one BSFW iteration runs them:
  (C, grad C) of the 50 atoms (render, blur, residual and criterion, adjoint, gradient
  sums), the grid certificate of the residual with its maximum, eta and its gradient at
  that maximum, and the weights-only LASSO of a 50-atom support whose last atom is new
  (columns of the other 49 come from the workspace cache, as in BSFW).
The metric counts the voxel x atom pairs of the (C, grad C) evaluation per step:
  value = 128 * 128 * 64 * 50 * steps / seconds / 1e9   [GVoxel*atom/s].
Inputs are built on the GPU before the timed region; every step runs in libsfw's kernels.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3   # vector and matrix FP32, dense
PEAK_HBM_GBS = 8000.0

# The dominant kernel: the certificate's inverse z pass, which multiplies the spectrum of q by
# every pair of table-kernel spectra and transforms along z (one launch per step, timed alone
# in the cert_zinv class). It is bound by HBM.
ROOF_CLASS = "cert_zinv"
ROOF_KERNEL = "k_fx_z_inverse (certificate: inverse z pass of every table-kernel pair)"

# Transform lengths of the library's fixed-length (two-stage) passes; the certificate grid
# takes the smallest of them >= max(n + R, 2R + 1) per axis when it is at most a quarter
# above the smallest 2-3-5-smooth length.
FIXED_LENGTHS = (16, 18, 20, 24, 25, 27, 30, 32, 36, 40, 45, 48, 50, 54, 60, 64, 72, 75, 80, 81,
                 90, 96, 100, 108, 120, 128, 135, 144, 150, 160, 180, 192, 225, 240, 256)

# Algorithmic ALU work per evaluated voxel-atom pair in FMA-slot units (one VALU instruction =
# 1 slot, one v_exp/v_log/v_rcp = 4 slots: quarter rate, measured), reported as 2 FLOP per slot.
RENDER_SLOTS_PER_PAIR = 4 + 3 * 4   # 4 VALU + log2, exp2, exp2
GRAD_SLOTS_PER_PAIR = 12 + 3 * 4    # 12 VALU + log2, exp2, exp2
SLOTS_PER_S = PEAK_FP32_TFLOPS * 1e12 / 2.0   # 256 CUs x 128 lanes x 2.4 GHz = 78.6 T slots/s

# Voxel boxes of one wave in the render and gradient kernels (x, y, z): a wave evaluates an atom
# only where its cut ball (the radius beyond which the atom is exactly zero in float32) meets its
# box; every other pair is an exact zero that it skips.
RENDER_WAVE_BOX = (16, 4, 4)
GRAD_WAVE_BOX = (16, 4, 16)
ETA_WAVE_BOX = (16, 4, 32)  # the one-launch eta kernel's 32-plane-deep tiles
ATOM_CUT_U = 110.0


def evaluated_pairs(shape, atoms, box):
    """Voxel-atom pairs the kernels evaluate: for every wave box (x, y, z) tiling the volume,
    box x * box y lanes (every lane computes, past the volume's edge too) x box z planes
    (clipped to the volume) per atom whose cut ball meets the box."""
    nz, ny, nx = shape
    bx, by, bz = box
    a = np.asarray(atoms, dtype=np.float64)
    r = a[:, 4] * (2.0 * ATOM_CUT_U) ** (1.0 / a[:, 5]) * 1.0001 + 1e-3
    total = 0
    for z0 in range(0, nz, bz):
        z1 = min(z0 + bz, nz) - 1
        dz = np.maximum(0.0, np.maximum(z0 - a[:, 3], a[:, 3] - z1))
        for y0 in range(0, ny, by):
            y1 = min(y0 + by, ny) - 1
            dy = np.maximum(0.0, np.maximum(y0 - a[:, 2], a[:, 2] - y1))
            x0 = np.arange(0, nx, bx, dtype=np.float64)
            x1 = np.minimum(x0 + bx, nx) - 1
            dx = np.maximum(0.0, np.maximum(x0[:, None] - a[None, :, 1], a[None, :, 1] - x1[:, None]))
            hit = dx * dx + (dy * dy + dz * dz)[None, :] <= (r * r)[None, :]
            total += int(hit.sum()) * bx * by * (z1 - z0 + 1)
    return total


# HBM traffic of one launch of the roofline kernel at this workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
#   bench.py --steps 2 --warmup 1 --profile-steps 0 --no-cpu-baseline --no-solve --proposal 0
#            --nnqp 0 --copy-probe-mib 256
# each scaled by the same counter's reading for the known 256 MiB device copy at the end.
# The record holds for the kernel source it was taken on: sha256 of the kernel's definition in
# KERNEL_SOURCE (from its template line to the next section rule). None until measured.
KERNEL_SOURCE = os.path.join(ROOT, "paper_2009_05473_amd", "csrc", "sfw_fft_fixed.hip")
KERNEL_START = ("template <int R1, int R2>\n__global__ __launch_bounds__(fx_threads(R1, R2)) "
                "void k_fx_z_inverse(")
SECTION_RULE = "\n// ----"
ROOF_TRAFFIC = {
    "fetch_kib": 13667.8, "write_kib": 68400.0,          # k_fx_z_inverse<9, 9>, per dispatch
    "copy_mib": 256, "copy_fetch_kib": 131087.8, "copy_write_kib": 262144.0,
    "source_sha256": "cefa6576c1d802f039c77da37a12c84e78561ebd27905bb7d9ada049af72d829",
}


def kernel_sha256():
    """sha256 of the roofline kernel's definition text (None if it cannot be located)."""
    import hashlib
    with open(KERNEL_SOURCE) as fh:
        src = fh.read()
    i = src.find(KERNEL_START)
    if i < 0:
        return None
    j = src.find(SECTION_RULE, i)
    return hashlib.sha256(src[i:j if j > 0 else len(src)].encode()).hexdigest()


def roof_traffic():
    """Counter-measured HBM bytes per launch of the roofline kernel, or None when the record
    is missing or the kernel source changed since it was taken."""
    t = ROOF_TRAFFIC
    if t is None:
        return None
    if kernel_sha256() != t["source_sha256"]:
        return None
    copy_bytes = float(t["copy_mib"]) * (1 << 20)
    fetch = t["fetch_kib"] * 1024.0 * copy_bytes / (t["copy_fetch_kib"] * 1024.0)
    write = t["write_kib"] * 1024.0 * copy_bytes / (t["copy_write_kib"] * 1024.0)
    return fetch + write


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=5,
                    help="untimed steps with every kernel class timed, for the breakdown")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the BSFW time-to-solution run after the timed steps")
    ap.add_argument("--batch", type=int, default=0, metavar="K",
                    help="also time sfw_solve_batch on the batched-solve workload, on one "
                         "workspace and on K workspaces (0: skip)")
    ap.add_argument("--batch-volumes", type=int, default=64)
    ap.add_argument("--proposal", type=int, default=3000, metavar="STEPS",
                    help="train the proposal network for STEPS steps, then compare BSFW with "
                         "learned and with grid seeds on held-out volumes (0: skip)")
    ap.add_argument("--proposal-volumes", type=int, default=10)
    ap.add_argument("--nnqp", type=int, default=4096, metavar="COUNT",
                    help="time sfw_nnqp_batch on COUNT weights QPs of 50 atoms in one launch, "
                         "and on one alone (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB on the device (the "
                         "known-size copy that scales the HBM counters of a --pmc run)")
    return ap.parse_args()


def cert_grid(shape, sigmas, ds, T=12.0):
    """Certificate transform lengths (x, y, z) and the largest table-kernel radius."""
    R = max(int(np.ceil(float(np.float32(s)) * (2 * T) ** (1 / float(d))))
            for s in sigmas for d in ds)

    def good(n):
        m = n
        while True:
            t = m
            for p in (2, 3, 5):
                while t % p == 0:
                    t //= p
            if t == 1:
                return m
            m += 1

    def length(nmin):
        g = good(nmin)
        for L in FIXED_LENGTHS:
            if nmin <= L <= g + g // 4:
                return L
        return g

    nz, ny, nx = shape
    return tuple(length(max(n + R, 2 * R + 1)) for n in (nx, ny, nz)), R


def zinv_bytes(shape, grid, npairs):
    """Algorithmic HBM bytes of one launch of the certificate's inverse z pass: the spectrum
    of q (Nx Ny Nz complex), the pair spectra (one octant each), and the z < nz planes of
    every pair's work array."""
    Nx, Ny, Nz = grid
    hx, hy, hz = Nx // 2 + 1, Ny // 2 + 1, Nz // 2 + 1
    nz = shape[0]
    return 8 * (Nx * Ny * Nz + npairs * hx * hy * hz + npairs * nz * Ny * Nx)


def cert_pass_bytes(shape, grid, npairs):
    """HBM bytes the certificate's other passes must move, each reading its input and writing
    its output once (the zinv_bytes convention): forward x (q in, full complex rows out), y and
    z passes; after the inverse z pass, the inverse y pass over every pair's z < nz planes and
    the x pass that reads them and keeps only block maxima."""
    Nx, Ny, Nz = grid
    nz, ny, nx = shape
    fx = 4 * nx * ny * nz + 8 * Nx * ny * nz          # x: q in, rows y < ny, z < nz out
    fy = 8 * Nx * ny * nz + 8 * Nx * Ny * nz          # y: all Ny rows out
    fz = 8 * Nx * Ny * nz + 8 * Nx * Ny * Nz          # z: all Nz planes out
    iy = npairs * 8 * (Nx * Ny * nz + Nx * ny * nz)   # inverse y: rows y < ny out
    ix = npairs * 8 * Nx * ny * nz                     # inverse x: read, maxima only
    return fx + fy + fz + iy + ix


COLUMN_CUT_U = 28.0


def column_box_voxels(shape, theta, psf_shape):
    """Voxels of a LASSO column's support box (host replica of the library's column box: the
    ball where the unit atom's u < 28, grown by one voxel and the PSF half-widths; x bounds
    widened to multiples of 4)."""
    m, sig, d = theta[:3], theta[3], theta[4]
    R = sig * (2.0 * COLUMN_CUT_U) ** (1.0 / d) + 1.0
    pz, py, px = psf_shape
    c = ((px - 1) / 2.0, (py - 1) / 2.0, (pz - 1) / 2.0)
    n = (shape[2], shape[1], shape[0])
    ext = []
    for a in range(3):
        lo = int(max(0.0, min(n[a], np.floor(m[a] - R - c[a]))))
        hi = int(max(0.0, min(n[a], np.ceil(m[a] + R + c[a]) + 1.0)))
        if a == 0:
            lo &= ~3
            hi = min(n[a], (hi + 3) & ~3)
        ext.append(max(hi - lo, 1))
    return ext[0] * ext[1] * ext[2]


def lut_taps(sigmas, ds, T=12.0):
    t = 0
    for s in sigmas:
        for d in ds:
            R = int(np.ceil(float(np.float32(s)) * (2 * T) ** (1 / float(d))))
            t += (2 * R + 1) ** 3
    return t


_ORACLE_SHARED = {}  # inputs of the parallel oracle leg, inherited by forked workers


def _render_chunk(atoms):
    import oracle
    return oracle.render(_ORACLE_SHARED["shape"], atoms)


def _grad_chunk(atoms):
    # dC/dw = lam (1 - eta(theta)), dC/dtheta = -w lam grad eta(theta): the sums of the analytic
    # gradient, per atom, on the shared q
    import oracle
    q, lam = _ORACLE_SHARED["q"], _ORACLE_SHARED["lam"]
    out = []
    for a in atoms:
        eta, g = oracle.eta_point(q, lam, a[1:6])
        out.append(np.concatenate([[lam * (1.0 - eta)], -a[0] * lam * g]))
    return out


def _oracle_step(oracle, prob, y, lam, atoms_eval, psf, cols, workers):
    """One step of the workload in the FP64 oracle: (C, grad C), grid certificate and its
    maximum, eta at the maximum, one new LASSO column with its Gram row and the NNLS. With
    workers > 1 the atoms are split into chunks rendered and differentiated by forked worker
    processes (the paper's parallelisation across atoms) and the Fourier-domain convolutions
    use `workers` FFT threads."""
    import multiprocessing as mp

    from scipy import fft as sfft
    from scipy import linalg, optimize
    cfg = prob.config
    with sfft.set_workers(workers):
        if workers == 1:
            _, _, _, q = oracle.criterion_and_grad(y, atoms_eval, psf, lam)
        else:
            ctx = mp.get_context("fork")
            chunks = np.array_split(atoms_eval, workers)
            _ORACLE_SHARED.update(shape=prob.shape)
            with ctx.Pool(workers) as pool:
                f = sum(pool.map(_render_chunk, chunks))
            r = y - oracle.blur(f, psf)
            0.5 * float(np.sum(r * r)) + lam * float(np.sum(atoms_eval[:, 0]))
            q = oracle.adjoint(r, psf)
            _ORACLE_SHARED.update(q=q, lam=lam)
            with ctx.Pool(workers) as pool:
                pool.map(_grad_chunk, chunks)
            _ORACLE_SHARED.clear()
        eta = oracle.grid_certificate(q, lam, cfg.sigma_grid, cfg.d_grid)
        _, (i, j, z, yy, x) = oracle.grid_argmax(eta)
        oracle.eta_point(q, lam, (x, yy, z, cfg.sigma_grid[i], cfg.d_grid[j]))
        a_new = oracle.lasso_columns(prob.shape, atoms_eval[-1:, 1:6], psf)
        A = np.vstack([cols, a_new])
        G = A @ A.T
        b = A @ y.reshape(-1)
        Lc = linalg.cholesky(G, lower=True)
        optimize.nnls(Lc.T, linalg.solve_triangular(Lc, b - lam, lower=True))


def cpu_baseline(prob, atoms_eval, psf, reps=3):
    """The oracle on one step of the same workload, from its own inputs: single thread (the
    correctness oracle as written) and on every core the process may use (atoms split across
    threads, multi-threaded FFTs). Median of `reps` steps each."""
    import oracle
    from paper_2009_05473_amd import synth
    from threadpoolctl import threadpool_limits
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(1):
        clean = oracle.blur(oracle.render(prob.shape, prob.atoms_true), psf)
        y = synth.make_observation(clean, prob.noise_unit, prob.config.noise_rel)
        lam = prob.config.lambda_rel * oracle.max_grid_certificate(
            y, psf, prob.config.sigma_grid, prob.config.d_grid)
        cols = oracle.lasso_columns(prob.shape, atoms_eval[:-1, 1:6], psf)  # cached in BSFW
    times = {}
    for threads in (1, cores):
        with threadpool_limits(threads):
            dts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                _oracle_step(oracle, prob, y, lam, atoms_eval, psf, cols, threads)
                dts.append(time.perf_counter() - t0)
        times[threads] = float(np.median(dts))
    V = int(np.prod(prob.shape))
    n = atoms_eval.shape[0]
    dt = times[cores]
    return {"value": V * n / dt / 1e9, "unit": "GVoxel*atom/s", "cores": cores, "kind": "oracle",
            "seconds": dt, "single_thread_value": V * n / times[1] / 1e9,
            "single_thread_seconds": times[1], "os_cpu_count": os.cpu_count(),
            "affinity_cores": cores,
            "sample": f"one full step of the same 128x128x64, 50-atom workload (float64 "
                      f"criterion and gradient, grid certificate and maximum, eta at the "
                      f"maximum, one new LASSO column with its Gram row and the NNLS), median "
                      f"of {reps}; value: {cores} cores (atoms split across forked worker "
                      f"processes, multi-threaded FFTs); single_thread_value: one thread"}


def solve_run(L, ws, H, Y, lam, prob, sg, dg):
    """Time-to-solution of sfw_solve (BSFW, grid proposal) on the same observation, from mu = 0,
    with the recovery of the true atoms (count, worst distance of a true centre to the nearest
    estimated one)."""
    import torch

    def timed(**kw):
        opts = L.default_options(mode="BSFW", sigma_grid=sg, d_grid=dg, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = L.sfw_solve(ws, Y, H, lam, opts)
        return (time.perf_counter() - t0,) + out

    # the first solve times the launch shapes; the reported time is the next one, and beside
    # it a solve with the default launch shapes and one replaying the chain from HIP graphs
    dt_first, _, st_first, _ = timed()
    dt, atoms, stats, code = timed()
    dt_eager, _, st_eager, _ = timed(autotune=0)
    dt_graph, _, st_graph, _ = timed(graphs=1)
    truth = prob.atoms_true
    err = max(float(np.min(np.linalg.norm(atoms[:, 1:4] - t[1:4], axis=1))) for t in truth) \
        if len(atoms) else float("inf")
    return {"workload": "128x128x64 volume, 50 true atoms, from mu = 0", "mode": "BSFW",
            "proposal": "grid", "seconds": dt, "status": int(code), "atoms_found": len(atoms),
            "atoms_true": int(truth.shape[0]), "max_centre_error_voxels": err,
            "iterations": stats["iterations"], "criterion": stats["criterion"],
            "eta_evaluations": stats["n_eval_eta"], "cgrad_evaluations": stats["n_eval_cgrad"],
            "ascent_iterations": stats["n_ascent_iterations"],
            "slide_iterations": stats["n_slide_iterations"],
            "seconds_certificate": stats["seconds_certificate"],
            "seconds_ascent": stats["seconds_ascent"], "seconds_lasso": stats["seconds_lasso"],
            "seconds_slide": stats["seconds_slide"],
            "seconds_first_solve": dt_first, "tunings_first_solve": st_first["n_tunings"],
            "seconds_default_shapes": dt_eager,
            "criterion_default_shapes": st_eager["criterion"],
            "seconds_graphs": dt_graph, "graph_replays": st_graph["n_graph_replays"],
            "criterion_graphs": st_graph["criterion"]}


def nnqp_run(L, count, k=50, reps=20):
    """Throughput of the batched weights QP (sfw_nnqp_batch): count problems of k atoms in one
    launch, and one problem alone (its latency). Each problem is G = A'A, c = A'y - 0.5 of a
    tall Gaussian A (2k + 8 rows) and y = A w + noise with a sparse non-negative w, 16 distinct
    seeded problems repeated; HIP events on torch's current stream bracket reps launches."""
    import torch
    rng = np.random.default_rng(5150)
    base = []
    for _ in range(16):
        A = rng.standard_normal((2 * k + 8, k))
        w = rng.uniform(0.2, 1.5, size=k) * (rng.uniform(size=k) < 0.7)
        y = A @ w + 0.3 * rng.standard_normal(A.shape[0])
        base.append((A.T @ A, A.T @ y - 0.5))
    rec = {"workload": f"weights QP, {k} atoms (Gram matrix of random columns)", "atoms": k}
    for n in (count, 1):
        G = torch.from_numpy(np.stack([base[i % 16][0] for i in range(n)])).cuda()
        c = torch.from_numpy(np.stack([base[i % 16][1] for i in range(n)])).cuda()
        w, info = L.sfw_nnqp_batch(G, c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            L.sfw_nnqp_batch(G, c, None, w, info)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        key = "batch" if n == count else "single"
        rec[key] = {"problems": n, "us_per_launch": us, "problems_per_s": n / us * 1e6,
                    "mean_passive_solves": float(info.float().mean().item())}
    return rec


def batch_run(L, synth, n_volumes, n_workspaces):
    """Throughput of sfw_solve_batch (BSFW, grid proposal) on the batched-solve workload
    (synth.draw_batch: volumes of 48..96 x 48..96 x 48 voxels holding 5..40 masses, each with
    its own PSF): the whole batch on one workspace (solves one after another), then on
    n_workspaces workspaces, each with its own stream (solves overlapping on the GPU). Both
    runs must return the same atoms."""
    import torch
    probs = synth.draw_batch(n_volumes)
    psf_max = tuple(max(p.config.psf_shape[a] for p in probs) for a in range(3))
    vol_max = tuple(max(p.config.shape[a] for p in probs) for a in range(3))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    data = []
    # inputs built on torch's current stream (the builder workspace's), which the tensor
    # arithmetic uses too
    with L.Workspace(vol_max, psf_max, 128) as builder:
        for p in probs:
            cfg = p.config
            H = dev(p.psf)
            clean = L.sfw_forward(builder, H, dev(p.atoms_true), p.shape)
            y = (clean + cfg.noise_rel * clean.max() * dev(p.noise_unit)).contiguous()
            _, best = L.sfw_certificate(builder, H, y, 1.0, list(np.float32(cfg.sigma_grid)),
                                        list(cfg.d_grid))
            data.append((y, H, float(np.float32(cfg.lambda_rel * best["eta"]))))
    streams = [torch.cuda.Stream() for _ in range(n_workspaces)]
    wss = [L.Workspace(vol_max, psf_max, 128, stream=st) for st in streams]
    cfg0 = probs[0].config
    opts = L.default_options(mode="BSFW", sigma_grid=[float(np.float32(v)) for v in cfg0.sigma_grid],
                             d_grid=cfg0.d_grid)
    torch.cuda.synchronize()
    print(f"[batch] {n_volumes} volumes built", file=sys.stderr, flush=True)
    L.sfw_solve_batch(wss, data[:n_workspaces], opts)  # untimed: first use of every workspace
    t0 = time.perf_counter()
    one = L.sfw_solve_batch(wss[:1], data, opts)
    t1 = time.perf_counter()
    print(f"[batch] one workspace: {t1 - t0:.3f} s", file=sys.stderr, flush=True)
    many = L.sfw_solve_batch(wss, data, opts)
    t2 = time.perf_counter()
    print(f"[batch] {n_workspaces} workspaces: {t2 - t1:.3f} s", file=sys.stderr, flush=True)
    # the same with the chain replayed from HIP graphs
    graphs = L.default_options(mode="BSFW", sigma_grid=[float(np.float32(v)) for v in cfg0.sigma_grid],
                               d_grid=cfg0.d_grid, graphs=1)
    t3 = time.perf_counter()
    replayed = L.sfw_solve_batch(wss, data, graphs)
    t4 = time.perf_counter()
    print(f"[batch] {n_workspaces} workspaces, graphs: {t4 - t3:.3f} s", file=sys.stderr, flush=True)
    for w in wss:
        w.close()
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(one, many))
    found = sum(len(r[0]) for r in many)
    true = sum(p.config.n_atoms for p in probs)
    return {"workload": f"{n_volumes} volumes of 48..96 x 48..96 x 48 voxels, 5..40 masses, "
                        "own Gaussian PSF each (up to 17x17x33), from mu = 0",
            "mode": "BSFW", "workspaces": n_workspaces,
            "voxels": int(sum(np.prod(p.config.shape) for p in probs)),
            "seconds_one_workspace": t1 - t0, "seconds": t2 - t1,
            "seconds_graphs": t4 - t3,
            "same_atoms_graphs": bool(all(np.array_equal(a[0], b[0]) for a, b in zip(many, replayed))),
            "volumes_per_s": n_volumes / (t2 - t1), "speedup": (t1 - t0) / (t2 - t1),
            "same_atoms": bool(same), "status_ok": int(sum(r[2] == L.SFW_OK for r in many)),
            "not_ok": {str(i): {"status": int(r[2]), "iterations": r[1]["iterations"],
                                "atoms": len(r[0]), "atoms_true": probs[i].config.n_atoms}
                       for i, r in enumerate(many) if r[2] != L.SFW_OK},
            "atoms_found": int(found), "atoms_true": int(true)}


def proposal_run(L, shape, steps, volumes):
    """Trains the proposal network on the GPU, then times BSFW from mu = 0 with learned and
    with grid seeds on held-out volumes. A Python-level failure is reported in the record."""
    from paper_2009_05473_amd import proposal
    rec = {"workload": f"{volumes} held-out 128x128x64 volumes, 50 atoms, BSFW from mu = 0",
           "train_steps": steps}
    try:
        with L.Net(shape) as net:
            net.set_params(proposal.init_params(np.random.default_rng(20000)))
            t0 = time.perf_counter()
            hist = proposal.train(L, net, steps, shape, seed=20000,
                                  log_every=max(1, steps // 5), log=sys.stderr)
            t_train = time.perf_counter() - t0
            rows = proposal.compare(L, net, proposal.held_out(volumes, shape), log=sys.stderr)
        rec.update({"train_seconds": t_train, "final_loss": hist[-1][1],
                    **proposal.summarize(rows)})
    except Exception as e:  # the main line still prints
        rec["error"] = f"{type(e).__name__}: {e}"
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); it has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2009_05473_amd import synth
    from paper_2009_05473_amd import _lib as L

    prob = synth.draw_problem("c3")
    cfg = prob.config
    shape = prob.shape
    V = int(np.prod(shape))
    N = cfg.n_atoms
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    psf = prob.psf.astype(np.float32)
    H = dev(psf)
    ws = L.Workspace(shape, psf.shape, 128)  # BSFW supports reach ~90 atoms before pruning
    sg = [float(np.float32(v)) for v in cfg.sigma_grid]
    dg = [float(v) for v in cfg.d_grid]

    # inputs: y = Phi mu* + noise on the GPU, lambda from the grid certificate of y
    clean = L.sfw_forward(ws, H, dev(prob.atoms_true.astype(np.float32)), shape)
    noise = dev(prob.noise_unit.astype(np.float32))
    Y = (clean + cfg.noise_rel * clean.max() * noise).contiguous()
    _, best0 = L.sfw_certificate(ws, H, Y, 1.0, sg, dg)
    lam = float(np.float32(cfg.lambda_rel * best0["eta"]))
    atoms_eval = synth.perturb(prob.atoms_true, prob.seed).astype(np.float32)
    A = dev(atoms_eval)
    R = torch.empty_like(Y)
    # one support per step: the 49 first atoms fixed, the last one new each step
    rng = np.random.default_rng(prob.seed + 900)
    supports = []
    for _ in range(args.warmup + args.profile_steps + args.steps):
        s = atoms_eval.copy()
        s[-1, 1:4] += rng.uniform(-1.0, 1.0, size=3).astype(np.float32)
        supports.append(dev(s))

    loss_buf = torch.empty(1, dtype=torch.float64, device="cuda")
    grad_buf = torch.empty((N, 6), dtype=torch.float32, device="cuda")
    w_buf = torch.empty(N, dtype=torch.float64, device="cuda")

    last_point = []

    def step(k):
        L.sfw_residual_grad(ws, H, Y, lam, A, r_out=R, loss_out=loss_buf, grad_out=grad_buf)  # a1-a5
        _, best = L.sfw_certificate(ws, H, None, lam, sg, dg, vol_shape=shape)  # a6-a7
        th = [[best["x"], best["y"], best["z"], sg[best["i_sigma"]], dg[best["i_d"]]]]
        last_point[:] = th
        L.sfw_eta_points(ws, shape, None, lam, th)                           # a8
        L.sfw_lasso_weights(ws, H, Y, lam, supports[k], w_out=w_buf)          # a9

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    # untimed: every kernel class behind an event pair, for the per-class breakdown
    prof = {}
    if args.profile_steps > 0:
        L.sfw_profile_begin(ws)
        for k in range(args.profile_steps):
            step(args.warmup + k)
        prof = L.sfw_profile_end(ws)
    # timed: only the roofline kernel carries events (its own start and stop, one launch a step)
    k0 = args.warmup + args.profile_steps
    torch.cuda.synchronize()
    L.sfw_profile_begin(ws, [ROOF_CLASS])
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k0 + k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    roof_prof = L.sfw_profile_end(ws)
    dt = t1 - t0
    ms_per_step = dt / args.steps * 1e3
    value = V * N * args.steps / dt / 1e9
    # untimed, with the breakdown: the (C, grad C) chain back to back, one event pair around 20
    # calls on the workspace's stream (torch's current one): its latency with the launch gaps,
    # without the device idle that an event pair around every kernel class adds
    chain_b2b_us = None
    if args.profile_steps > 0:
        chain_reps = 20
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0.record()
        for _ in range(chain_reps):
            L.sfw_residual_grad(ws, H, Y, lam, A, r_out=R, loss_out=loss_buf, grad_out=grad_buf)
        c1.record()
        torch.cuda.synchronize()
        chain_b2b_us = c0.elapsed_time(c1) * 1e3 / chain_reps

    # algorithmic work per launch of each kernel class: HBM bytes that the operation must move
    # (its inputs and outputs, not the implementation's intermediate arrays) and ALU slots of
    # the voxel-atom pairs the kernels evaluate (host replica of their box test)
    px, py, pz = psf.shape[2], psf.shape[1], psf.shape[0]
    taps = px * py * pz
    conv_flops = 2.0 * V * taps
    grid, rmax = cert_grid(shape, sg, dg)
    npairs = (len(sg) * len(dg) + 1) // 2
    zbytes = zinv_bytes(shape, grid, npairs)
    pairs_render = evaluated_pairs(shape, atoms_eval, RENDER_WAVE_BOX)
    pairs_grad = evaluated_pairs(shape, atoms_eval, GRAD_WAVE_BOX)
    vb = 4.0 * V  # one float32 volume
    # the step's eta point (the certificate maximum's unit atom) and new LASSO column (the
    # support's last atom, moved every step)
    pairs_eta = evaluated_pairs(shape, [[1.0] + list(last_point[0])], ETA_WAVE_BOX)
    col_vox = column_box_voxels(shape, [float(v) for v in atoms_eval[-1, 1:6]], psf.shape)
    nd = N  # Gram row against the support's columns and y
    work = {  # class: (HBM bytes, ALU slots) per launch
        "render": (vb + 32.0 * N, float(pairs_render * RENDER_SLOTS_PER_PAIR)),
        "conv_residual": (3 * vb, 0.0),   # f and y in, r out (r stays in LDS for the adjoint)
        "conv_adjoint": (vb, 0.0),        # q out
        "grad": (vb, float(pairs_grad * GRAD_SLOTS_PER_PAIR)),  # q in
        "cert_zinv": (float(zbytes), 0.0),
        "cert_fft": (cert_pass_bytes(shape, grid, npairs) / 2.0, 0.0),  # two launches a step
        "eta_grad": (0.0, float(pairs_eta * GRAD_SLOTS_PER_PAIR)),
        # the new column over its box: one FMA slot per tap per box voxel (the atom's own
        # evaluation on the block tiles aside)
        "lasso_conv": (4.0 * col_vox, float(col_vox * taps)),
        # the Gram row: the new column and nd + 1 others (columns, y) over its box
        "lasso_dots": (4.0 * col_vox * (nd + 2), 0.0),
    }
    ps = max(args.profile_steps, 1)
    breakdown = {}
    step_ms = sum(ms for _, ms in prof.values()) / ps if prof else 0.0
    for name, (launches, ms) in prof.items():
        e = {"launches_per_step": launches / ps, "ms_per_step": ms / ps,
             "us_per_launch": ms / launches * 1e3, "share": (ms / ps) / step_ms}
        t = ms / launches * 1e-3
        if name in work:
            nbytes, slots = work[name]
            t_hbm, t_alu = nbytes / (PEAK_HBM_GBS * 1e9), slots / SLOTS_PER_S
            bound = "hbm" if t_hbm >= t_alu else "alu"
            e.update({"bound": bound, "bytes": nbytes, "alu_slots": slots,
                      "roofline_us": max(t_hbm, t_alu) * 1e6,
                      "frac": max(t_hbm, t_alu) / t})
        if name in ("conv_residual", "conv_adjoint"):
            # spectral blur: the direct convolution's FLOP rate it stands in for
            e["direct_equivalent_tflops"] = conv_flops / t / 1e12
        breakdown[name] = e
    if prof:
        chain = ("prep", "render", "conv_residual", "conv_adjoint", "grad", "grad_finalize")
        fwd_grad_ms = sum(prof.get(k, (0, 0.0))[1] for k in chain) / ps
        roof_us = sum(breakdown[k].get("roofline_us", 0.0) for k in chain if k in breakdown)
        breakdown["fwd_grad_GVoxel_atom_per_s"] = V * N / (fwd_grad_ms * 1e-3) / 1e9
        breakdown["fwd_grad_chain"] = {
            "us": fwd_grad_ms * 1e3, "roofline_us": roof_us, "frac": roof_us / (fwd_grad_ms * 1e3),
            "us_back_to_back": chain_b2b_us, "frac_back_to_back": roof_us / chain_b2b_us,
            "GVoxel_atom_per_s_back_to_back": V * N / (chain_b2b_us * 1e-6) / 1e9,
            "evaluated_pairs_render": pairs_render, "evaluated_pairs_grad": pairs_grad,
            "nominal_pairs": V * N,
            "definition": "sum over the chain's kernel classes of max(algorithmic HBM bytes / "
                          "8 TB/s, ALU slots of evaluated voxel-atom pairs / 78.6 T slots/s), "
                          "over the measured chain time: us = the classes' event-timed sums, "
                          "us_back_to_back = 20 chains between one event pair"}

    # roofline of the dominant kernel, timed live over the timed region
    launches, ms = roof_prof[ROOF_CLASS]
    avg_s = ms / launches * 1e-3
    achieved = zbytes / avg_s / 1e9
    roofline = {"kernel": ROOF_KERNEL, "bound": "hbm", "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": roof_traffic(), "us_per_launch": avg_s * 1e6,
                "bytes_per_launch": zbytes, "grid": list(grid), "pairs": npairs}

    out = {
        "metric": "fwd+grad GVoxel*atom/s (one step = every hot-path row once)",
        "value": value,
        "unit": "GVoxel*atom/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128x128x64 volume, 50 atoms, 9x9x15 Gaussian PSF, 4x3 "
                               "certificate grid (BSFW iteration)",
                   "volume": [128, 128, 64], "atoms": N, "psf": [px, py, pz],
                   "grid": [len(sg), len(dg)], "lambda": lam, "parallelism": "none"},
        "roofline": roofline,
        "breakdown": breakdown,
    }
    if not args.no_solve:
        out["solve"] = solve_run(L, ws, H, Y, lam, prob, sg, dg)
    if args.batch > 0:
        out["batch"] = batch_run(L, synth, args.batch_volumes, args.batch)
    if args.proposal > 0:
        out["proposal"] = proposal_run(L, shape, args.proposal, args.proposal_volumes)
    if args.nnqp > 0:
        out["nnqp"] = nnqp_run(L, args.nnqp)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, atoms_eval.astype(np.float64),
                                           psf.astype(np.float64))
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    ws.close()


if __name__ == "__main__":
    main()
