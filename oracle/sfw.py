"""Plain FP64 implementation of what the BSFW / SFW hot path computes.

TEST INFRASTRUCTURE ONLY (see the package docstring): slow, obviously correct,
NumPy/SciPy in float64, no blocking or fusion beyond what the definitions say.

Notation (paper, section 1): an atom is theta = (m, sigma, d) with weight w,
G(theta, w; s) = w exp(-||m - s||^d / (2 sigma^d)); the measure is
mu = sum_n w_n delta_{theta_n}; the observation is y = H * sum_n G(theta_n, w_n) + eps.

Conventions (readings where the paper is silent, listed in the design notes):
  * volumes are ``[nz][ny][nx]`` arrays, voxel centres at integer coordinates,
    unit spacing, Euclidean distance in voxel units;
  * atoms are rows ``(w, mx, my, mz, sigma, d)``;
  * H * f is the zero-padded linear convolution with output on the volume grid
    ("same"), the PSF being odd-sized and centred at (P-1)/2;
  * Phi^T r is the exact adjoint: correlation with H, zero outside.

Pins (tests/test_oracle_*.py): every function below is pinned against closed
forms, invariants, brute force or library special cases. The solver loop's
choice among local optima (which the paper leaves to "e.g. BFGS") is
parity unpinned beyond the end-to-end recovery properties.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import fft as sfft
from scipy import linalg, optimize

T_TRUNC = 12.0  # grid kernels keep every voxel of the cube holding g >= exp(-T)
PRUNE_REL = 1e-6  # "remove zero-weighted masses": w <= PRUNE_REL * max(w)
# The loop continues while eta* > 1. After the LASSO every atom of the support has
# eta = 1 exactly (its KKT condition), so in floating point the test needs a margin.
ETA_TOL = 1e-3
# Two masses closer than this in every coordinate of (m, sigma, d) are one mass.
MERGE_TOL = 5e-2

__all__ = [
    "T_TRUNC", "PRUNE_REL", "ETA_TOL", "MERGE_TOL", "merge_coincident", "coords", "atom_profile", "render", "blur", "adjoint",
    "criterion", "criterion_and_grad", "forward_vjp", "eta_point", "lut_radius", "lut_kernel",
    "grid_certificate", "grid_argmax", "lasso_columns", "lasso_weights", "nnqp", "ascent",
    "slide", "prune", "solve", "SolveResult", "max_grid_certificate",
]


# ---------------------------------------------------------------- operators

def coords(shape):
    """Voxel centre coordinates (x, y, z) broadcastable over ``[nz][ny][nx]`` (section 1.1, s in R^3)."""
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return x, y, z


def atom_profile(shape, mx, my, mz, sigma, d):
    """Unit-weight generalized isotropic Gaussian on every voxel.

    Section 1.1, definition of the atom G: exp(-||m - s||^d / (2 sigma^d)).
    """
    x, y, z = coords(shape)
    r = np.sqrt((x - mx) ** 2 + (y - my) ** 2 + (z - mz) ** 2)
    return np.exp(-(r ** d) / (2.0 * sigma ** d))


def render(shape, atoms):
    """sum_n G(theta_n, w_n; s) over every voxel, no truncation (section 1.1, observation model)."""
    f = np.zeros(shape, dtype=np.float64)
    for w, mx, my, mz, s, d in np.asarray(atoms, dtype=np.float64).reshape(-1, 6):
        f += w * atom_profile(shape, mx, my, mz, s, d)
    return f


def _check_psf(psf):
    if psf.ndim != 3 or any(p % 2 == 0 for p in psf.shape):
        raise ValueError("PSF must be 3-D with odd sizes")


def _linear_conv_same(vol, ker):
    """Zero-padded linear convolution, cropped to vol's grid with the kernel centred.

    Computed through the Fourier domain as the paper does (section 2, implementation
    points): both operands are zero-padded to at least the full linear size, so the
    circular product equals the linear one.
    """
    n = vol.shape
    p = ker.shape
    full = [n[i] + p[i] - 1 for i in range(3)]
    fs = [sfft.next_fast_len(s, real=True) for s in full]
    spec = sfft.rfftn(vol, fs) * sfft.rfftn(ker, fs)
    out = sfft.irfftn(spec, fs)
    c = [(pi - 1) // 2 for pi in p]
    return np.ascontiguousarray(out[c[0]:c[0] + n[0], c[1]:c[1] + n[1], c[2]:c[2] + n[2]])


def blur(f, psf):
    """Phi applied to a rendered volume: (H * f)(s) = sum_t H[c + t] f(s - t), f = 0 off the grid.

    Section 1.1, observation model with the PSF.
    """
    psf = np.asarray(psf, dtype=np.float64)
    _check_psf(psf)
    return _linear_conv_same(np.asarray(f, dtype=np.float64), psf)


def adjoint(r, psf):
    """Phi^T on volumes: q(s) = sum_t H[c + t] r(s + t), zero outside (section 1.2, certificate)."""
    psf = np.asarray(psf, dtype=np.float64)
    _check_psf(psf)
    return _linear_conv_same(np.asarray(r, dtype=np.float64), psf[::-1, ::-1, ::-1])


def criterion(y, atoms, psf, lam):
    """C = 1/2 ||y - Phi mu||^2 + lam * sum_n w_n (section 1.2, criterion C). Returns (C, r)."""
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    y = np.asarray(y, dtype=np.float64)
    r = y - blur(render(y.shape, atoms), psf)
    return 0.5 * float(np.sum(r * r)) + lam * float(np.sum(atoms[:, 0])), r


def _atom_terms(shape, mx, my, mz, s, d):
    """Per-voxel pieces of one atom: (dx, dy, dz, r2, u, g, mask r2 > 0)."""
    x, y, z = coords(shape)
    dx = np.broadcast_to(x - mx, shape)
    dy = np.broadcast_to(y - my, shape)
    dz = np.broadcast_to(z - mz, shape)
    r2 = dx * dx + dy * dy + dz * dz
    r = np.sqrt(r2)
    u = r ** d / (2.0 * s ** d)
    g = np.exp(-u)
    return dx, dy, dz, r2, u, g, r2 > 0


def criterion_and_grad(y, atoms, psf, lam):
    """(C, dC/d(w, mx, my, mz, sigma, d) per atom, r, q).

    Section 2 says the gradient of C is computed analytically. With
    q = Phi^T (y - Phi mu), u = ||s - m||^d / (2 sigma^d), g = exp(-u):
      dC/dw     = lam - sum q g
      dC/dm     = -w d sum q g u (s - m) / ||s - m||^2
      dC/dsigma = -w (d / sigma) sum q g u
      dC/dd     =  w sum q g u ln(||s - m|| / sigma)
    Voxels at the atom centre contribute 0 to the m, sigma and d terms (limits).
    """
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    y = np.asarray(y, dtype=np.float64)
    C, r = criterion(y, atoms, psf, lam)
    q = adjoint(r, psf)
    grad = np.zeros_like(atoms)
    for n, (w, mx, my, mz, s, d) in enumerate(atoms):
        dx, dy, dz, r2, u, g, nz = _atom_terms(y.shape, mx, my, mz, s, d)
        qg = q * g
        qgu = qg * u
        inv_r2 = np.where(nz, 1.0 / np.where(nz, r2, 1.0), 0.0)
        log_rs = np.where(nz, 0.5 * np.log(np.where(nz, r2, 1.0)) - math.log(s), 0.0)
        grad[n, 0] = lam - qg.sum()
        grad[n, 1] = -w * d * np.sum(qgu * dx * inv_r2)
        grad[n, 2] = -w * d * np.sum(qgu * dy * inv_r2)
        grad[n, 3] = -w * d * np.sum(qgu * dz * inv_r2)
        grad[n, 4] = -w * (d / s) * qgu.sum()
        grad[n, 5] = w * np.sum(qgu * log_rs)
    return C, grad, r, q


def forward_vjp(g, atoms, psf):
    """Vector-Jacobian product of the forward model: d<g, Phi mu>/d(w, mx, my, mz, sigma, d).

    Section 1.1 observation model, differentiated as in section 2 (analytic derivatives).
    <g, H * f> = <Phi^T g, f>, so with q = Phi^T g and f = sum_n w_n exp(-u_n):
      d/dw     = sum q g
      d/dm     = w d sum q g u (s - m) / ||s - m||^2
      d/dsigma = w (d / sigma) sum q g u
      d/dd     = -w sum q g u ln(||s - m|| / sigma)
    with the centre voxel contributing 0 to the m, sigma and d terms (limits).
    """
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    g = np.asarray(g, dtype=np.float64)
    q = adjoint(g, psf)
    out = np.zeros_like(atoms)
    for n, (w, mx, my, mz, s, d) in enumerate(atoms):
        dx, dy, dz, r2, u, gn, nz = _atom_terms(g.shape, mx, my, mz, s, d)
        qg = q * gn
        qgu = qg * u
        inv_r2 = np.where(nz, 1.0 / np.where(nz, r2, 1.0), 0.0)
        log_rs = np.where(nz, 0.5 * np.log(np.where(nz, r2, 1.0)) - math.log(s), 0.0)
        out[n, 0] = qg.sum()
        out[n, 1] = w * d * np.sum(qgu * dx * inv_r2)
        out[n, 2] = w * d * np.sum(qgu * dy * inv_r2)
        out[n, 3] = w * d * np.sum(qgu * dz * inv_r2)
        out[n, 4] = w * (d / s) * qgu.sum()
        out[n, 5] = -w * np.sum(qgu * log_rs)
    return out


def eta_point(q, lam, theta):
    """Certificate at one point of the domain and its gradient in (mx, my, mz, sigma, d).

    Section 1.2: eta = Phi^T (y - Phi mu) / lam, i.e. the correlation of the residual
    with a blurred unit atom at theta, which equals (1/lam) sum_s g(s; theta) q(s)
    with q = H-correlated residual.
    """
    mx, my, mz, s, d = [float(v) for v in theta]
    dx, dy, dz, r2, u, g, nz = _atom_terms(q.shape, mx, my, mz, s, d)
    qg = q * g
    qgu = qg * u
    inv_r2 = np.where(nz, 1.0 / np.where(nz, r2, 1.0), 0.0)
    log_rs = np.where(nz, 0.5 * np.log(np.where(nz, r2, 1.0)) - math.log(s), 0.0)
    eta = qg.sum() / lam
    grad = np.array([
        d * np.sum(qgu * dx * inv_r2),
        d * np.sum(qgu * dy * inv_r2),
        d * np.sum(qgu * dz * inv_r2),
        (d / s) * qgu.sum(),
        -np.sum(qgu * log_rs),
    ]) / lam
    return float(eta), grad


# ---------------------------------------------------------------- grid certificate

def lut_radius(sigma, d, T=T_TRUNC):
    """Half-width R of the cube holding every voxel with g >= exp(-T): R = ceil(sigma (2T)^(1/d))."""
    return int(math.ceil(sigma * (2.0 * T) ** (1.0 / d)))


def lut_kernel(sigma, d, T=T_TRUNC):
    """Unit atom centred on a voxel, tabulated on [-R, R]^3 (section 2, lookup table for eta)."""
    R = lut_radius(sigma, d, T)
    t = np.arange(-R, R + 1, dtype=np.float64)
    r = np.sqrt(t[:, None, None] ** 2 + t[None, :, None] ** 2 + t[None, None, :] ** 2)
    return np.exp(-(r ** d) / (2.0 * sigma ** d))


def grid_certificate(q, lam, sigma_grid, d_grid, T=T_TRUNC):
    """eta on the candidate grid: voxel centres x sigma_grid x d_grid, shape ``[ns][nd][nz][ny][nx]``.

    Section 1.3, step 1 (a maximum attained on a grid) with the lookup table of
    section 2: eta_ij(m) = (1/lam) sum_{||t||_inf <= R_ij} LUT_ij[t] q(m + t).
    """
    q = np.asarray(q, dtype=np.float64)
    out = np.zeros((len(sigma_grid), len(d_grid)) + q.shape)
    for i, s in enumerate(sigma_grid):
        for j, d in enumerate(d_grid):
            lut = lut_kernel(s, d, T)
            # correlation = convolution with the flipped table
            out[i, j] = _linear_conv_same(q, lut[::-1, ::-1, ::-1]) / lam
    return out


def grid_argmax(eta):
    """(max value, i_sigma, i_d, z, y, x) of eta; ties go to the lowest C-order flat index.

    Section 1.3, step 1: the maximum of eta itself (mu is a positive measure).
    """
    flat = int(np.argmax(eta))  # numpy returns the first occurrence
    idx = np.unravel_index(flat, eta.shape)
    return float(eta.reshape(-1)[flat]), tuple(int(v) for v in idx)


def max_grid_certificate(y, psf, sigma_grid, d_grid, T=T_TRUNC):
    """max over the grid of Phi^T y (lam = 1), the scale used to set lam in the workloads."""
    q = adjoint(y, psf)
    return grid_argmax(grid_certificate(q, 1.0, sigma_grid, d_grid, T))[0]


# ---------------------------------------------------------------- LASSO on weights

def lasso_columns(shape, thetas, psf):
    """Columns a_n = H * g(theta_n) for unit-weight atoms, stacked as ``[k][V]``."""
    thetas = np.asarray(thetas, dtype=np.float64).reshape(-1, 5)
    return np.stack([blur(atom_profile(shape, *th), psf).reshape(-1) for th in thetas]) \
        if len(thetas) else np.zeros((0, int(np.prod(shape))))


def lasso_weights(y, thetas, psf, lam):
    """argmin_{w >= 0} 1/2 ||y - sum_n w_n a_n||^2 + lam sum_n w_n (section 1.3, step 3).

    With G = A^T A and b = A^T y the objective is 1/2 w^T G w - (b - lam 1)^T w + const,
    minimised by nnqp. Returns (w, G, b).
    """
    y = np.asarray(y, dtype=np.float64)
    A = lasso_columns(y.shape, thetas, psf)
    k = A.shape[0]
    if k == 0:
        return np.zeros(0), np.zeros((0, 0)), np.zeros(0)
    G = A @ A.T
    b = A @ y.reshape(-1)
    return nnqp(G, b - lam), G, b


def nnqp(G, c):
    """argmin_{w >= 0} 1/2 w^T G w - c^T w: the weights step of section 1.3 (step 3) once the
    Gram matrix G = A^T A of the columns and c = A^T y - lam are formed.

    With G = L L^T the objective is 1/2 ||L^T w - L^{-1} c||^2 + const, a non-negative
    least-squares problem handed to scipy.optimize.nnls.
    """
    G = np.asarray(G, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    k = c.shape[0]
    if k == 0:
        return np.zeros(0)
    try:
        L = linalg.cholesky(G, lower=True)
    except linalg.LinAlgError:
        # duplicate atoms make G singular; any KKT point is then a minimiser
        L = linalg.cholesky(G + 1e-12 * np.trace(G) / k * np.eye(k), lower=True)
    rhs = linalg.solve_triangular(L, c, lower=True)
    w, _ = optimize.nnls(L.T, rhs, maxiter=50 * k + 100)
    return w


# ---------------------------------------------------------------- local ascent / descent

def _theta_bounds(shape, bounds):
    nz, ny, nx = shape
    slo, shi = bounds["sigma"]
    dlo, dhi = bounds["d"]
    return [(0.0, nx - 1.0), (0.0, ny - 1.0), (0.0, nz - 1.0), (slo, shi), (dlo, dhi)]


def ascent(q, lam, theta0, shape, bounds, gtol=1e-9, ftol=1e-12, maxiter=200):
    """Step 1: local ascent of eta over the box of the domain from the grid maximum.

    The paper says "e.g. BFGS"; a box-bounded quasi-Newton method (L-BFGS-B) is used.
    Returns (theta*, eta*).
    """
    b = _theta_bounds(shape, bounds)
    x0 = np.clip(np.asarray(theta0, dtype=np.float64), [lo for lo, _ in b], [hi for _, hi in b])

    def fun(th):
        e, g = eta_point(q, lam, th)
        return -e, -g

    res = optimize.minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=b,
                            options={"gtol": gtol, "ftol": ftol, "maxiter": maxiter})
    th = res.x
    return th, eta_point(q, lam, th)[0]


def slide(y, atoms, psf, lam, bounds, gtol=1e-9, ftol=1e-12, maxiter=1000):
    """Local descent of C on all (w, theta) from the current measure (SFW step 4, BSFW step 2b).

    Box-bounded quasi-Newton (L-BFGS-B), weights bounded below by 0.
    """
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    k = atoms.shape[0]
    if k == 0:
        return atoms.copy()
    tb = _theta_bounds(y.shape, bounds)
    b = []
    for _ in range(k):
        b.append((0.0, None))
        b.extend(tb)

    def fun(x):
        C, g, _, _ = criterion_and_grad(y, x.reshape(k, 6), psf, lam)
        return C, g.reshape(-1)

    lo = np.array([v[0] if v[0] is not None else -np.inf for v in b])
    hi = np.array([v[1] if v[1] is not None else np.inf for v in b])
    x0 = np.clip(atoms.reshape(-1), lo, hi)
    res = optimize.minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=b,
                            options={"gtol": gtol, "ftol": ftol, "maxiter": maxiter})
    return res.x.reshape(k, 6)


def merge_coincident(atoms, tol=MERGE_TOL):
    """Fuse masses sitting at the same point of the domain into one Dirac.

    w_i delta_theta + w_j delta_theta is the single mass (w_i + w_j) delta_theta;
    points closer than ``tol`` in every coordinate of (m, sigma, d) count as one.
    Atoms are visited in order; each joins the first earlier kept atom it
    coincides with, whose parameters become the weight-averaged ones.
    """
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    kept = []
    for a in atoms:
        for b in kept:
            if np.max(np.abs(a[1:6] - b[1:6])) <= tol:
                wsum = a[0] + b[0]
                if wsum > 0:
                    b[1:6] = (b[0] * b[1:6] + a[0] * a[1:6]) / wsum
                b[0] = wsum
                break
        else:
            kept.append(a.copy())
    return np.array(kept).reshape(-1, 6)


def prune(atoms, rel=PRUNE_REL, tol=MERGE_TOL):
    """Remove zero-weighted masses and update the measure (SFW step 5, BSFW steps 4 and 3b).

    Keeps w > rel * max w, then merges coincident masses (``merge_coincident``).
    """
    atoms = np.asarray(atoms, dtype=np.float64).reshape(-1, 6)
    if atoms.shape[0] == 0:
        return atoms
    wmax = atoms[:, 0].max()
    if wmax <= 0:
        return atoms[:0]
    return merge_coincident(atoms[atoms[:, 0] > rel * wmax], tol)


# ---------------------------------------------------------------- solver loop

@dataclass
class SolveResult:
    atoms: np.ndarray
    converged: bool
    iterations: int
    criterion: float
    history: list = field(default_factory=list)


def solve(y, psf, lam, sigma_grid, d_grid, bounds, mode="BSFW", max_iter=200, T=T_TRUNC,
          eta_tol=ETA_TOL, ascent_opts=None, slide_opts=None, log=None):
    """SFW (algorithm 1) or BSFW (algorithm 2) from mu = 0.

    Each iteration: residual of the current measure, certificate grid maximum,
    local ascent of eta; if eta* > 1 the support grows, the weights are re-fitted
    by the LASSO and zero weights are pruned (SFW also slides all parameters
    before pruning). Otherwise BSFW runs its single final slide and prune and
    both variants stop. Stopping uses eta* <= 1 + eta_tol (the paper's "> 1" continues).
    ``log``, if given, is called with each iteration's history entry (progress only).
    """
    if mode not in ("BSFW", "SFW"):
        raise ValueError("mode must be 'BSFW' or 'SFW'")
    ascent_opts = ascent_opts or {}
    slide_opts = slide_opts or {}
    y = np.asarray(y, dtype=np.float64)
    atoms = np.zeros((0, 6))
    history = []
    for k in range(1, max_iter + 1):
        C, r = criterion(y, atoms, psf, lam)
        q = adjoint(r, psf)
        eta = grid_certificate(q, lam, sigma_grid, d_grid, T)
        gmax, (i, j, z, yy, x) = grid_argmax(eta)
        theta0 = np.array([x, yy, z, sigma_grid[i], d_grid[j]], dtype=np.float64)
        theta, eta_star = ascent(q, lam, theta0, y.shape, bounds, **ascent_opts)
        history.append({"k": k, "C": C, "grid_max": gmax, "eta_star": eta_star,
                        "n_atoms": atoms.shape[0]})
        if log is not None:
            log(history[-1])
        if eta_star <= 1.0 + eta_tol:
            if mode == "BSFW":
                atoms = prune(slide(y, atoms, psf, lam, bounds, **slide_opts))
            Cf, _ = criterion(y, atoms, psf, lam)
            return SolveResult(atoms, True, k, Cf, history)
        thetas = np.vstack([atoms[:, 1:6], theta[None, :]])
        w, _, _ = lasso_weights(y, thetas, psf, lam)
        atoms = np.hstack([w[:, None], thetas])
        if mode == "SFW":
            atoms = slide(y, atoms, psf, lam, bounds, **slide_opts)
        atoms = prune(atoms)
    Cf, _ = criterion(y, atoms, psf, lam)
    return SolveResult(atoms, False, max_iter, Cf, history)
