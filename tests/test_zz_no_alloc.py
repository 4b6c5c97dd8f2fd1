"""dipole_readout_noalloc, the readout for callers that cannot allocate:
through the C-ABI, its per-molecule outputs and ensemble sums equal those of
dipole_readout bit for bit, on two calls in a row (the second on a smaller
batch, so the static scratch holds the first call's partials when the second
starts), and a batch beyond its static scratch is rejected before any
launch."""

import ctypes as C

import numpy as np
import pytest
import torch

from gpu_helpers import banner
from workloads import get_config
from workloads.molecule_inputs import potentials

pytestmark = pytest.mark.gpu


def _outputs(n, nc):
    mk = lambda *s: torch.full(s, np.nan, dtype=torch.float64, device="cuda")  # noqa: E731
    return (mk(n, nc) if nc == 3 else mk(n)), mk(n), mk(n), mk(nc + 2)


@pytest.mark.parametrize("basis,j_max", [("m0", 10), ("jm", 2)])
def test_noalloc_readout_equals_dipole_readout(basis, j_max):
    from paper_2209_04487_amd import msqd
    n_big, n_small = 5000, 1500                  # 5 blocks, then 2 (a ragged tail each)
    cfg = get_config("cfg0", j_max=j_max, basis=basis, n_r=128)
    banner(f"dipole_readout_noalloc {basis} j_max={j_max}: {n_big} then {n_small} molecules")
    mols = msqd.Molecules(n_big, cfg.n_r, j_max, cfg.r_min, cfg.r_max, cfg.mass, cfg.dt_au,
                          *potentials(cfg), np.ones(cfg.n_r), prec="fp32", basis=basis)
    rng = np.random.default_rng(7)
    psi = rng.standard_normal(tuple(mols.psi.shape) + (2,)).astype(np.float32)
    mols.psi.copy_(torch.view_as_complex(torch.as_tensor(psi)).cuda())
    mols.absorbed.copy_(torch.as_tensor(rng.uniform(0, 1e-2, n_big)))
    nc = mols.n_sums - 2
    for n in (n_big, n_small):
        d = msqd.qd_desc.from_buffer_copy(mols.desc)
        d.n_mol = n
        ref = _outputs(n, nc)
        got = _outputs(n, nc)
        msqd.dipole_readout(d, mols.ws, mols.psi, mols.absorbed, *ref)
        msqd.dipole_readout_noalloc(d, mols.ws, mols.psi, mols.absorbed, *got)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert torch.isfinite(got[3]).all()
        # and the sums are the sums of the per-molecule values
        dd = got[0].cpu().numpy().reshape(n, nc)
        np.testing.assert_allclose(got[3].cpu().numpy()[:nc], dd.sum(axis=0), rtol=1e-12,
                                   atol=1e-12 * np.abs(dd).sum())


def test_noalloc_readout_rejects_batches_beyond_its_scratch():
    """n_mol above 1024 x 1024 with sums: MSQD_EUNSUP, checked on the host
    before any launch (the device pointers are never touched); without sums
    the limit does not apply."""
    from paper_2209_04487_amd import msqd
    d = msqd.qd_desc(1024 * 1024 + 1, 256, 10, msqd.FP32, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, 0)
    fake = C.c_void_p(1 << 20)
    rc = msqd.lib.dipole_readout_noalloc(C.byref(d), fake, fake, fake, fake, fake, fake, fake, None)
    assert rc == msqd.MSQD_EUNSUP
    assert "1048576" in msqd.last_error()
