"""Model curves sampled on the radial grid and the initial wavefunction.

The radial grid is periodic: r_k = r_min + k dr, dr = (r_max - r_min) / n_r,
with r_max itself excluded.
"""

from __future__ import annotations

import math

import numpy as np

from .configs import Config


def r_grid(cfg: Config) -> np.ndarray:
    dr = (cfg.r_max - cfg.r_min) / cfg.n_r
    return cfg.r_min + dr * np.arange(cfg.n_r, dtype=np.float64)


def potentials(cfg: Config):
    """(U_g, U_e, mu12) on the grid, hartree / e a0.

    Ground state: Morse D (1 - exp(-a (r - r_e)))^2 (optionally shifted by -D,
    the form of the paper's Eq. (6)); excited: c0 + c1 exp(-b (r - r0)), the
    repulsive form of Eq. (7); transition dipole exp(-mu_b (r - mu_r0)^2).
    """
    r = r_grid(cfg)
    ug = cfg.morse_d * (1.0 - np.exp(-cfg.morse_a * (r - cfg.morse_re))) ** 2
    if cfg.morse_shift:
        ug = ug - cfg.morse_d
    ue = cfg.ue_c0 + cfg.ue_c1 * np.exp(-cfg.ue_b * (r - cfg.ue_r0))
    mu = np.exp(-cfg.mu_b * (r - cfg.mu_r0) ** 2)
    return ug, ue, mu


def morse_v0(cfg: Config) -> np.ndarray:
    """Closed-form Morse v = 0 function on the grid, discretely normalised so
    that sum |psi|^2 dr = 1 (real, float64 [n_r])."""
    r = r_grid(cfg)
    lam = math.sqrt(2.0 * cfg.mass * cfg.morse_d) / cfg.morse_a
    y = cfg.morse_a * (r - cfg.morse_re)
    logpsi = -(lam - 0.5) * y - lam * np.exp(-y)
    logpsi -= logpsi.max()
    psi = np.exp(logpsi)
    dr = (cfg.r_max - cfg.r_min) / cfg.n_r
    psi /= math.sqrt(np.sum(psi * psi) * dr)
    return psi


def block_cell_list(cfg) -> np.ndarray:
    """Flat E_x index of each molecule for the block placement: one molecule
    per cell of the cube [lo, lo+n)^3, i fastest (int32)."""
    n = cfg.block_n
    out = np.empty(n ** 3, dtype=np.int32)
    idx = 0
    for k in range(cfg.block_lo, cfg.block_lo + n):
        for j in range(cfg.block_lo, cfg.block_lo + n):
            for i in range(cfg.block_lo, cfg.block_lo + n):
                out[idx] = (k * cfg.ny + j) * cfg.nx + i
                idx += 1
    return out


def bloch_parameters(cfg: Config):
    """Two-level parameters of the workload's molecule with its ro-vibrations
    frozen at r_e: (omega0, mu) in atomic units, omega0 the vertical gap
    U_e(r_e) - U_g(r_e) and mu = mu12(r_e) / sqrt(3), the J = 0 -> 1 matrix
    element of cos(theta) times the transition dipole."""
    re = cfg.morse_re
    ug = 0.0 if not cfg.morse_shift else -cfg.morse_d
    ue = cfg.ue_c0 + cfg.ue_c1 * math.exp(-cfg.ue_b * (re - cfg.ue_r0))
    mu = math.exp(-cfg.mu_b * (re - cfg.mu_r0) ** 2) / math.sqrt(3.0)
    return ue - ug, mu
