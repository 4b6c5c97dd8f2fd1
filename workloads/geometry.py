"""Voxelised material maps, one uint8 id per E-component location.

The Yee placement used throughout: E_x at (i+1/2, j, k), E_y at (i, j+1/2, k),
E_z at (i, j, k+1/2) in cell units; arrays are stored [component][k][j][i].
A location belongs to a shape when its coordinates fall in the shape's
half-open intervals.
"""

from __future__ import annotations

import math

import numpy as np

from .configs import MAT_GLASS, MAT_METAL, MAT_VACUUM, Config

# offsets (x, y, z) of the three E components inside a cell
E_OFFSETS = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))


def _coords(cfg: Config, comp: int):
    ox, oy, oz = E_OFFSETS[comp]
    x = np.arange(cfg.nx, dtype=np.float64) + ox
    y = np.arange(cfg.ny, dtype=np.float64) + oy
    z = np.arange(cfg.nz, dtype=np.float64) + oz
    return x, y, z


def _srr_mask_xy(cfg: Config, x, y):
    """Square split ring centred in each unit cell, gap cut in the +y arm."""
    g = cfg.geom
    cell, outer, arm, gap = g["cell"], g["outer"], g["arm"], g["gap"]
    lo = (cell - outer) / 2.0
    hi = lo + outer
    ilo, ihi = lo + arm, hi - arm
    glo = (cell - gap) / 2.0
    ghi = glo + gap
    X = np.mod(x, cell)[None, :]
    Y = np.mod(y, cell)[:, None]
    in_outer = (X >= lo) & (X < hi) & (Y >= lo) & (Y < hi)
    in_inner = (X >= ilo) & (X < ihi) & (Y >= ilo) & (Y < ihi)
    in_gap = (X >= glo) & (X < ghi) & (Y >= ihi) & (Y < hi)
    return in_outer & ~in_inner & ~in_gap


def _hole_mask_xy(cfg: Config, x, y):
    """Equilateral triangles (one side along x, apex towards +y) at the given
    centroids; True inside a hole."""
    g = cfg.geom
    side = g["side"]
    h = side * math.sqrt(3.0) / 2.0
    X = x[None, :]
    Y = y[:, None]
    mask = np.zeros((len(y), len(x)), dtype=bool)
    for cx, cy in g["centres"]:
        ybase = cy - h / 3.0
        yapex = cy + 2.0 * h / 3.0
        inside = (Y >= ybase) & (Y < yapex) & (np.abs(X - cx) < (yapex - Y) / math.sqrt(3.0))
        mask |= inside
    return mask


def material_map(cfg: Config) -> np.ndarray:
    """uint8 [3][nz][ny][nx] material ids for the workload's geometry."""
    mat = np.zeros((3, cfg.nz, cfg.ny, cfg.nx), dtype=np.uint8)
    if cfg.geometry == "vacuum":
        return mat
    g = cfg.geom
    for comp in range(3):
        x, y, z = _coords(cfg, comp)
        glass_z = z >= g["glass_k"]
        mat[comp][glass_z] = MAT_GLASS
        metal_z = (z >= g["z0"]) & (z < g["z1"])
        if cfg.geometry == "srr":
            xy = _srr_mask_xy(cfg, x, y)
        elif cfg.geometry == "nanohole":
            xy = ~_hole_mask_xy(cfg, x, y)
        else:
            raise ValueError(cfg.geometry)
        sel = metal_z[:, None, None] & xy[None, :, :]
        mat[comp][sel] = MAT_METAL
    return mat


def eps_table(cfg: Config) -> np.ndarray:
    """Relative permittivity (eps_inf for the metal) per material id."""
    t = np.ones(3, dtype=np.float64)
    t[MAT_VACUUM] = 1.0
    t[MAT_GLASS] = cfg.eps_glass
    t[MAT_METAL] = cfg.eps_inf
    return t
