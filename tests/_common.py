"""Helpers shared by the tests: tolerances and seeded problems (no method arithmetic here)."""
import numpy as np

from paper_2009_05473_amd import synth


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def rel_err(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)


def config_problem(name, rep=0):
    return synth.draw_problem(name, rep)


def parity_atoms(prob):
    """Perturbed (non-stationary) parameters near the truth, as float32-representable values."""
    a = synth.perturb(prob.atoms_true, prob.seed)
    return a.astype(np.float32).astype(np.float64)
