"""The algorithmic per-unit counts behind bench.py's roofline figures, pinned
to their definitions (CPU): bytes are the state read and written once plus
the small per-molecule or per-cell terms, and the molecular flop count
follows the stated recipe (5 N log2 N per complex FFT, 6 per phase multiply,
14 per rotation point)."""

import math

import bench
from workloads import get_config


def test_molecular_step_bytes():
    cfg = get_config("cfg2")
    psi = 2 * 11 * 256 * 8                       # 2 states x 11 J x 256 r, complex64
    assert bench.mol_bytes_per_step(cfg, "mixed") == 2 * psi + 4 + 4 + 16 + 8 + 8 == 90152
    assert bench.mol_bytes_per_step(get_config("cfg1"), "fp64") == 2 * 2 * psi + 8 + 4 + 16 + 8 + 8 == 180268


def test_molecular_step_flops():
    cfg = get_config("cfg2")
    n, nj = 256, 11
    fft = 5 * n * int(math.log2(n))
    lines = 2 * nj
    expect = lines * (4 * fft + 4 * 6 * n) + nj * n * 14 + 2 * nj * n * 3 + (nj - 1) * n * 8
    assert bench.mol_flops_per_step(cfg) == expect
    assert abs(expect / 1e6 - 1.113) < 0.001


def test_jm_counts():
    assert bench.jm_bytes_per_step(256) == 2 * 8 * 256 * 8 + 64 == 32832
    assert bench.jmg_bytes_per_step(256, 5) == 2 * 2 * 36 * 256 * 8 + 64 == 294976
    assert abs(bench.jmg_flops_per_step(256, 5) / 1e6 - 6.00) < 0.01


def test_stencil_bytes():
    assert bench.stencil_bytes_per_cell("mixed") == 18 * 4 + 3 == 75
    assert bench.stencil_bytes_per_cell("fp64") == 18 * 8 + 3 == 147
    assert bench.stencil_min_bytes_per_cell("mixed") == 12 * 4 + 3 == 51
