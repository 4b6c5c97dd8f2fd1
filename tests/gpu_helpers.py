"""Shared helpers for the GPU parity tests (seeded inputs only)."""

import math
import sys

import numpy as np


def banner(msg):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def model_arrays(n_r, r_min=1.0, r_max=12.0):
    r = r_min + (r_max - r_min) / n_r * np.arange(n_r)
    ug = 0.17 * (1.0 - np.exp(-(r - 2.0))) ** 2
    ue = 0.17 + 0.30 * np.exp(-1.2 * (r - 2.0))
    mu = np.exp(-0.1 * (r - 2.0) ** 2)
    return r, ug, ue, mu


def random_state(seed, n_mol, n_j, n_r, dr):
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal((n_mol, 2, n_j, n_r)) + 1j * rng.standard_normal((n_mol, 2, n_j, n_r))
    nrm = np.sqrt(np.sum(np.abs(psi) ** 2, axis=(1, 2, 3)) * dr)
    return psi / nrm[:, None, None, None]


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


TOL = {"fp64": 1e-11, "fp32": 3e-5, "mixed": 3e-5}

__all__ = ["banner", "model_arrays", "random_state", "rel_err", "TOL", "math"]
