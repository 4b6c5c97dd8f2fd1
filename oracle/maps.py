"""Oracle: molecule placement -> Yee cell -> compressed list of occupied cells.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper spreads the molecules of the layer evenly over all processors and
sends each one the local field of its grid point (section "Efficient
numerical implementation ...", molecular mapping).  On one device this is a
flat molecule-major batch; what remains is the integer map from molecule to
the E_x edge it samples and deposits on, and the cells grouped so that the
per-cell dipole sum has a fixed order.

Placement uses integers only: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
draws three 64-bit words per molecule, and cell = ((u >> 11) * N) >> 53 with
an exact wide product.
"""

from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)


def scale_index(u: int, n: int) -> int:
    """floor(((u >> 11) / 2^53) * n), exactly, with integers only."""
    return ((u >> 11) * n) >> 53


def slab_cells(seed, n_mol, nx, ny, k0, nk):
    """Flat E_x index (k*ny + j)*nx + i of each molecule, uniform over the
    slab k in [k0, k0+nk), all i, j."""
    rng = SplitMix64(seed)
    cells = np.empty(n_mol, dtype=np.int64)
    for m in range(n_mol):
        ux = rng.next()
        uy = rng.next()
        uz = rng.next()
        i = scale_index(ux, nx)
        j = scale_index(uy, ny)
        k = k0 + scale_index(uz, nk)
        cells[m] = (k * ny + j) * nx + i
    return cells


def block_cells(n_per_side, lo, nx, ny):
    """One molecule per cell of the cube [lo, lo+n)^3, i fastest."""
    n = n_per_side
    cells = np.empty(n ** 3, dtype=np.int64)
    for m in range(n ** 3):
        i = lo + m % n
        j = lo + (m // n) % n
        k = lo + m // (n * n)
        cells[m] = (k * ny + j) * nx + i
    return cells


def csr(cell_of_mol):
    """(occ_cell, occ_ptr, mol_perm): occupied cells in increasing order,
    offsets into mol_perm, and the molecules listed cell by cell, in
    increasing molecule index inside each cell."""
    cell_of_mol = np.asarray(cell_of_mol, dtype=np.int64)
    perm = np.argsort(cell_of_mol, kind="stable")
    occ, counts = np.unique(cell_of_mol, return_counts=True)
    ptr = np.zeros(len(occ) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    return occ, ptr, perm


def cells_from_config(cfg):
    if cfg.placement == "block":
        return block_cells(cfg.block_n, cfg.block_lo, cfg.nx, cfg.ny)
    return slab_cells(cfg.seed, cfg.n_mol, cfg.nx, cfg.ny, cfg.slab_k0, cfg.slab_nk)
