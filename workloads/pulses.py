"""Incident-pulse samples E_inc(t_{n+1/2}) in V/m, and the seeded knot draw."""

from __future__ import annotations

import math

import numpy as np

from . import units as U
from .configs import Config

_MASK64 = (1 << 64) - 1


def splitmix64_stream(seed: int, count: int) -> list[int]:
    """SplitMix64 outputs (Steele, Lea and Flood 2014) for a seed; used only to
    draw seeded input values (the knot amplitudes)."""
    out = []
    s = seed & _MASK64
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & _MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out.append(z ^ (z >> 31))
    return out


def knot_values(cfg: Config) -> np.ndarray:
    """64 envelope knots a_j = (0.5 + u_j) 1e-3 au, u_j = (x >> 11) 2^-53."""
    xs = splitmix64_stream(cfg.knot_seed, cfg.n_knots)
    u = np.array([(x >> 11) * 2.0 ** -53 for x in xs], dtype=np.float64)
    return (0.5 + u) * 1.0e-3


def knot_times(cfg: Config) -> np.ndarray:
    t_run = cfg.n_steps * cfg.dt
    return np.arange(cfg.n_knots, dtype=np.float64) * t_run / (cfg.n_knots - 1)


def envelope_basis(cfg: Config, t: np.ndarray) -> np.ndarray:
    """Hat functions h_j(t) of the piecewise-linear envelope, shape [len(t), n_knots]."""
    tk = knot_times(cfg)
    h = np.zeros((len(t), cfg.n_knots))
    for j in range(cfg.n_knots):
        e = np.zeros(cfg.n_knots)
        e[j] = 1.0
        h[:, j] = np.interp(t, tk, e)
    return h


def source_times(cfg: Config, n0: int, n_steps: int) -> np.ndarray:
    """Half-step times t_{n+1/2} at which the source sheet is sampled."""
    return (np.arange(n0, n0 + n_steps, dtype=np.float64) + 0.5) * cfg.dt


def source_values(cfg: Config, n0: int = 0, n_steps: int | None = None,
                  knots: np.ndarray | None = None, omega: float | None = None) -> np.ndarray:
    """E_inc at t_{n+1/2} (V/m) for steps n0 .. n0+n_steps-1."""
    if n_steps is None:
        n_steps = cfg.n_steps
    t = source_times(cfg, n0, n_steps)
    w = cfg.omega if omega is None else omega
    if cfg.pulse == "gauss":
        tau = cfg.fwhm_fs * U.FS
        env = cfg.e0_au * U.E_AU * np.exp(-4.0 * math.log(2.0) * (t - cfg.t0) ** 2 / tau ** 2)
        return env * np.cos(w * (t - cfg.t0))
    if cfg.pulse == "knots":
        a = knot_values(cfg) if knots is None else np.asarray(knots, dtype=np.float64)
        env = np.interp(t, knot_times(cfg), a) * U.E_AU
        return env * np.cos(w * t)
    if cfg.pulse == "cw":
        # continuous wave switched on smoothly over the first cw_ramp_fs
        t_on = cfg.cw_ramp_fs * U.FS
        ramp = np.where(t < t_on, np.sin(0.5 * np.pi * np.clip(t, 0.0, None) / t_on) ** 2, 1.0)
        return cfg.e0_au * U.E_AU * ramp * np.cos(w * t)
    raise ValueError(cfg.pulse)


def source_jacobian(cfg, n0: int, n_steps: int, knots=None, omega=None) -> np.ndarray:
    """d E_inc(t_{n+1/2}) / d p for the knot envelope E_inc = A(t) cos(omega t):
    rows p = knot_0 .. knot_{K-1} (per au of field) then omega (per rad/s);
    shape [n_knots + 1, n_steps], V/m per parameter unit."""
    t = source_times(cfg, n0, n_steps)
    a = knot_values(cfg) if knots is None else np.asarray(knots, dtype=np.float64)
    w = cfg.omega if omega is None else omega
    h = envelope_basis(cfg, t)
    jac = np.zeros((cfg.n_knots + 1, n_steps))
    jac[:cfg.n_knots] = (h * np.cos(w * t)[:, None]).T * U.E_AU
    jac[cfg.n_knots] = -(h @ a) * t * np.sin(w * t) * U.E_AU
    return jac
