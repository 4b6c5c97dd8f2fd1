"""The gradient of the differentiation workload at its own parameters (one SRR
cell 96 x 96 x 80, 20,000 molecules, N_r = 128, J <= 6, the 64-knot envelope
drawn from its seed, the 0.10 Eh carrier, all 4,000 steps, a checkpoint
every 200): the FP32 gradient against the FP64 one.

Here the pulse barely excites the molecules: the FP64 yield is about 9e-11,
below what FP32 resolves (FP32 round-off of the ground state's tail beyond
r_diss reads about 2e-10), so the yields are not compared.  The gradient is
a linear propagation of the adjoint and is resolved: FP32 and FP64 agree to
about 1e-4 (largest knot difference over the largest knot component, and
the carrier derivative).  Tolerance 1e-3."""

import numpy as np
import pytest
import torch

from gpu_helpers import banner
from workloads import get_config
from workloads.pulses import knot_values

pytestmark = pytest.mark.gpu


def test_workload_gradient_fp32_against_fp64():
    from paper_2209_04487_amd.grad import yield_and_gradient
    cfg = get_config("cfg3")
    assert cfg.n_steps == 4000 and cfg.ckpt_every == 200
    banner(f"differentiation workload gradient fp32 vs fp64: {cfg.n_mol} molecules, {cfg.n_steps} steps")
    kn = knot_values(cfg)
    Y64, dk64, dw64 = yield_and_gradient(cfg, kn, cfg.omega, prec="fp64")
    torch.cuda.empty_cache()
    Y32, dk32, dw32 = yield_and_gradient(cfg, kn, cfg.omega, prec="fp32")
    torch.cuda.empty_cache()
    print(f"Y fp64 {Y64:.4e} fp32 {Y32:.4e}; |dk| {np.linalg.norm(dk64):.4e}; dY/dw {dw64:.4e}")
    assert 0.0 < Y64 < 1e-9
    assert np.abs(dk64).max() > 0 and dw64 != 0.0
    assert np.abs(dk32 - dk64).max() <= 1e-3 * np.abs(dk64).max()
    assert abs(dw32 - dw64) <= 1e-3 * abs(dw64)
