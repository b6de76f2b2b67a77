"""Seeded synthetic workloads for the 3D deconvolution problem.

This module only draws inputs: atom parameters, the point spread function and a
unit-variance noise volume. It holds none of the solver's arithmetic, so the
FP64 oracle and the GPU library can both be fed from it without sharing any
computation. Building the observation y = Phi mu* + noise needs the forward
model, which the caller supplies (``make_observation``).

The paper's own experiment (section 3) uses a tomographic diffractive
microscopy PSF that is not available; the configurations below stand in for
it with an anisotropic Gaussian PSF that is, like the paper's, invariant by
rotation about the optical (z) axis and much wider along z.

Conventions shared with the library and the oracle:
  * volumes are C-order float arrays ``[nz][ny][nx]`` (x fastest);
  * voxel centres sit at integer coordinates, unit spacing on every axis;
  * an atom is a row ``(w, mx, my, mz, sigma, d)`` in voxel units;
  * the PSF is ``[Pz][Py][Px]`` with odd sizes, centred at ``(P-1)/2``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

ATOM_FIELDS = ("w", "mx", "my", "mz", "sigma", "d")

# Box of the parameter domain (the paper only says sigma, d > 0; these bounds
# are the reading used by both the oracle and the library).
SIGMA_BOUNDS = (0.5, 4.0)
D_BOUNDS = (1.2, 3.0)


@dataclass(frozen=True)
class Config:
    name: str
    shape: tuple  # (nz, ny, nx)
    n_atoms: int
    sigma_range: tuple
    d_range: tuple  # (lo, hi); lo == hi means a fixed exponent
    w_range: tuple
    margin: float  # centres drawn uniformly in [margin, n - margin] per axis
    min_spacing: float
    psf_sigma_xy: float
    psf_sigma_z: float
    psf_shape: tuple  # (Pz, Py, Px)
    noise_rel: float  # noise std = noise_rel * max(Phi mu*)
    sigma_grid: tuple
    d_grid: tuple = (1.5, 2.0, 2.5)
    lambda_rel: float = 0.05  # lambda = lambda_rel * max over the grid of Phi^T y


CONFIGS = {
    # small case: 32^3, 3 atoms, d = 2
    "c1": Config("c1", (32, 32, 32), 3, (1.0, 2.0), (2.0, 2.0), (1.0, 2.0), 6.0, 3.0,
                 1.0, 2.0, (15, 9, 9), 0.01, tuple(np.linspace(1.0, 2.0, 4))),
    # 64x64x32, 10 atoms, free exponent, wide PSF (6,975 taps)
    "c2": Config("c2", (32, 64, 64), 10, (0.8, 2.5), (1.5, 2.5), (0.5, 2.0), 6.0, 3.0,
                 1.5, 3.5, (31, 15, 15), 0.02, tuple(np.linspace(0.8, 2.5, 4))),
    # 128x128x64, 50 atoms, the throughput workload
    "c3": Config("c3", (64, 128, 128), 50, (1.0, 2.0), (2.0, 2.0), (1.0, 2.0), 6.0, 3.0,
                 1.0, 2.0, (15, 9, 9), 0.01, tuple(np.linspace(1.0, 2.0, 4))),
}

CONFIG_INDEX = {"c1": 1, "c2": 2, "c3": 3}


def seed_for(config: str, rep: int = 0) -> int:
    """Seed = 1000 * config number + repetition."""
    return 1000 * CONFIG_INDEX[config] + rep


def gaussian_psf(sigma_xy: float, sigma_z: float, shape: tuple) -> np.ndarray:
    """Anisotropic Gaussian PSF ``[Pz][Py][Px]`` (odd sizes), normalised to unit sum."""
    pz, py, px = shape
    if pz % 2 == 0 or py % 2 == 0 or px % 2 == 0:
        raise ValueError("PSF sizes must be odd")
    z = np.arange(pz) - (pz - 1) / 2
    y = np.arange(py) - (py - 1) / 2
    x = np.arange(px) - (px - 1) / 2
    gz = np.exp(-0.5 * (z / sigma_z) ** 2)
    gy = np.exp(-0.5 * (y / sigma_xy) ** 2)
    gx = np.exp(-0.5 * (x / sigma_xy) ** 2)
    h = gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return h / h.sum()


def draw_centres(rng: np.random.Generator, n: int, shape: tuple, margin: float,
                 min_spacing: float, max_tries: int = 100000) -> np.ndarray:
    """Centres (mx, my, mz) drawn one at a time, redrawn while closer than min_spacing."""
    nz, ny, nx = shape
    lo = np.array([margin, margin, margin])
    hi = np.array([nx - margin, ny - margin, nz - margin])
    out = np.zeros((n, 3))
    k = 0
    tries = 0
    while k < n:
        c = rng.uniform(lo, hi)
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place centres with the requested spacing")
        if k and np.min(np.linalg.norm(out[:k] - c, axis=1)) < min_spacing:
            continue
        out[k] = c
        k += 1
    return out


def draw_atoms(cfg: Config, rng: np.random.Generator) -> np.ndarray:
    """Ground-truth atoms ``[N][6]``; draw order: centres, sigma, d, w."""
    n = cfg.n_atoms
    m = draw_centres(rng, n, cfg.shape, cfg.margin, cfg.min_spacing)
    sigma = rng.uniform(*cfg.sigma_range, size=n)
    if cfg.d_range[0] == cfg.d_range[1]:
        d = np.full(n, cfg.d_range[0])
    else:
        d = rng.uniform(*cfg.d_range, size=n)
    w = rng.uniform(*cfg.w_range, size=n)
    atoms = np.zeros((n, 6))
    atoms[:, 0] = w
    atoms[:, 1:4] = m
    atoms[:, 4] = sigma
    atoms[:, 5] = d
    return atoms


def perturb(atoms: np.ndarray, seed: int) -> np.ndarray:
    """Parity point near the truth: dm ~ U[-.5,.5]^3, sigma*U[.9,1.1], d+U[-.1,.1], w*U[.8,1.2]."""
    rng = np.random.default_rng(seed + 500)
    a = np.array(atoms, dtype=np.float64, copy=True)
    n = a.shape[0]
    a[:, 1:4] += rng.uniform(-0.5, 0.5, size=(n, 3))
    a[:, 4] *= rng.uniform(0.9, 1.1, size=n)
    a[:, 5] += rng.uniform(-0.1, 0.1, size=n)
    a[:, 0] *= rng.uniform(0.8, 1.2, size=n)
    return a


def random_atoms(rng: np.random.Generator, n: int, shape: tuple, sigma_range=(0.8, 2.5),
                 d_range=(1.3, 2.8), w_range=(0.5, 2.0), margin: float = 0.0) -> np.ndarray:
    """Unstructured atoms for operator tests (centres anywhere in the box, no spacing rule)."""
    nz, ny, nx = shape
    a = np.zeros((n, 6))
    a[:, 0] = rng.uniform(*w_range, size=n)
    a[:, 1] = rng.uniform(margin, max(nx - 1 - margin, margin), size=n)
    a[:, 2] = rng.uniform(margin, max(ny - 1 - margin, margin), size=n)
    a[:, 3] = rng.uniform(margin, max(nz - 1 - margin, margin), size=n)
    a[:, 4] = rng.uniform(*sigma_range, size=n)
    a[:, 5] = rng.uniform(*d_range, size=n)
    return a


@dataclass
class Problem:
    config: Config
    seed: int
    atoms_true: np.ndarray  # [N][6] float64
    psf: np.ndarray  # [Pz][Py][Px] float64, unit sum
    noise_unit: np.ndarray  # [nz][ny][nx] float64, N(0, 1)
    bounds: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.config.shape


def draw_problem(config: str, rep: int = 0) -> Problem:
    """Draw one seeded problem; draw order: centres, sigma, d, w, noise."""
    return _draw(CONFIGS[config], seed_for(config, rep))


def experiment_config(n: int, n_atoms: int) -> Config:
    """The paper's SFW / BSFW comparison (section 3): an n^3 volume (60 to 100) holding 4, 6 or 8
    masses under Gaussian noise. The 32^3 workload's atom distributions, PSF, noise level,
    lambda rule and grid stand in for the paper's unavailable PSF and data."""
    return replace(CONFIGS["c1"], name=f"x{n}_{n_atoms}", shape=(n, n, n), n_atoms=n_atoms)


def draw_experiment(n: int, n_atoms: int, rep: int) -> Problem:
    """One seeded problem of the comparison; seed = 10^6 + 10^4 n + 100 n_atoms + rep (rep < 100)."""
    if not 0 <= rep < 100 or not 0 < n_atoms < 100:
        raise ValueError("rep must be in [0, 100) and n_atoms in [1, 100)")
    return _draw(experiment_config(n, n_atoms), 10 ** 6 + 10 ** 4 * n + 100 * n_atoms + rep)


def draw_held_out(index: int, shape: tuple = (64, 128, 128), n_atoms: int = 50) -> Problem:
    """Held-out problem ``index`` of the learned-proposal comparison: the 128x128x64 workload's
    distributions (or another shape / atom count), seed 5000 + index, draw_problem's order."""
    if index < 0:
        raise ValueError("index must be >= 0")
    cfg = replace(CONFIGS["c3"], shape=tuple(shape), n_atoms=int(n_atoms))
    return _draw(cfg, 5000 + index)


BATCH_SHAPES_XY = tuple(range(48, 97, 8))  # n_x, n_y of a batch volume; n_z = 48


def batch_config(rng: np.random.Generator, index: int) -> Config:
    """One volume of the batched-solve workload (many uneven small volumes), drawn in the order
    n_x, n_y, N, PSF sigma_xy, PSF sigma_z: n_x, n_y in {48, 56, ..., 96}, n_z = 48,
    N ~ U{5..40}, the 64x64x32 workload's atom distributions, noise and grid, and an
    anisotropic Gaussian PSF with sigma_xy ~ U[1, 2], sigma_z ~ U[2, 4] cut at
    ceil(4 sigma) per axis (P_xy <= 17, P_z <= 33)."""
    nx = int(rng.choice(BATCH_SHAPES_XY))
    ny = int(rng.choice(BATCH_SHAPES_XY))
    n_atoms = int(rng.integers(5, 41))
    sxy = float(rng.uniform(1.0, 2.0))
    sz = float(rng.uniform(2.0, 4.0))
    hxy, hz = int(np.ceil(4.0 * sxy)), int(np.ceil(4.0 * sz))
    return replace(CONFIGS["c2"], name=f"b{index}", shape=(48, ny, nx), n_atoms=n_atoms,
                   psf_sigma_xy=sxy, psf_sigma_z=sz, psf_shape=(2 * hz + 1, 2 * hxy + 1, 2 * hxy + 1))


def draw_batch(n_volumes: int = 64, rep: int = 0) -> list:
    """The batched-solve workload: n_volumes seeded problems. Volume i draws its shape, N and PSF
    from seed s = 4000 + 100 rep + i (batch_config), then its atoms and noise from seed
    s + 100000 in draw_problem's order."""
    if not 0 <= n_volumes <= 100:
        raise ValueError("n_volumes must be in [0, 100]")
    out = []
    for i in range(n_volumes):
        seed = 4000 + 100 * rep + i
        cfg = batch_config(np.random.default_rng(seed), i)
        out.append(_draw(cfg, seed + 10 ** 5))
    return out


def _draw(cfg: Config, seed: int) -> Problem:
    rng = np.random.default_rng(seed)
    atoms = draw_atoms(cfg, rng)
    noise = rng.standard_normal(cfg.shape)
    psf = gaussian_psf(cfg.psf_sigma_xy, cfg.psf_sigma_z, cfg.psf_shape)
    nz, ny, nx = cfg.shape
    bounds = {"m_lo": (0.0, 0.0, 0.0), "m_hi": (nx - 1.0, ny - 1.0, nz - 1.0),
              "sigma": SIGMA_BOUNDS, "d": D_BOUNDS}
    return Problem(cfg, seed, atoms, psf, noise, bounds)


def make_observation(clean: np.ndarray, noise_unit: np.ndarray, noise_rel: float) -> np.ndarray:
    """y = clean + noise_rel * max(clean) * noise_unit, where ``clean`` is Phi mu* from the caller's forward model."""
    clean = np.asarray(clean, dtype=np.float64)
    if noise_rel == 0.0:
        return clean.copy()
    return clean + noise_rel * float(clean.max()) * noise_unit
