"""Pins of the oracle's integer placement maps."""

import random
from fractions import Fraction

import numpy as np

from oracle.maps import SplitMix64, block_cells, csr, scale_index, slab_cells


def test_splitmix64_known_answer():
    """First output for seed 0 of the published SplitMix64 generator (equal to
    the first nextLong() of Java's SplittableRandom(0))."""
    assert SplitMix64(0).next() == 0xE220A8397B1DCDAF


def test_scale_index_is_exact_floor():
    rnd = random.Random(7)
    for _ in range(2000):
        u = rnd.getrandbits(64)
        n = rnd.randrange(1, 5000)
        exact = int(Fraction(u >> 11, 2 ** 53) * n)        # floor of a positive rational
        assert scale_index(u, n) == exact
    assert scale_index((1 << 64) - 1, 192) == 191


def test_block_cells_cover_the_block():
    cells = block_cells(4, 10, 24, 24)
    assert len(set(cells.tolist())) == 64
    k, rem = np.divmod(cells, 24 * 24)
    j, i = np.divmod(rem, 24)
    assert set(i.tolist()) == set(j.tolist()) == set(k.tolist()) == {10, 11, 12, 13}
    assert i[0] == 10 and i[1] == 11 and j[4] == 11 and k[16] == 11


def test_slab_cells_range_and_uniformity():
    nx, ny, k0, nk = 24, 20, 5, 3
    cells = slab_cells(3, 20000, nx, ny, k0, nk)
    k, rem = np.divmod(cells, nx * ny)
    j, i = np.divmod(rem, nx)
    assert i.min() >= 0 and i.max() < nx and j.min() >= 0 and j.max() < ny
    assert k.min() >= k0 and k.max() < k0 + nk
    counts = np.bincount(i, minlength=nx)
    expect = 20000 / nx
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 3 * nx


def test_csr_structure():
    cells = slab_cells(11, 5000, 16, 16, 0, 4)
    occ, ptr, perm = csr(cells)
    assert np.all(np.diff(occ) > 0)
    assert ptr[0] == 0 and ptr[-1] == len(cells)
    assert sorted(perm.tolist()) == list(range(len(cells)))
    for c in range(len(occ)):
        members = perm[ptr[c]:ptr[c + 1]]
        assert np.all(cells[members] == occ[c])
        assert np.all(np.diff(members) > 0)
