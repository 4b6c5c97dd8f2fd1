"""GPU parity of the field solver (fdtd_step, monitor, flux_readout) with the
FP64 oracle: all six field components, the Drude currents and the CPML
auxiliaries after the run, on the tiny vacuum grid and on one SRR unit cell
of the silver array (metal, glass, both CPMLs, source, monitor).

FP64 tolerance 1e-11 relative to the largest field value; FP32 2e-4."""

import numpy as np
import pytest
import torch

from gpu_helpers import banner, rel_err
from oracle.fdtd import FluxMonitor, yee_from_config
from workloads import get_config
from workloads.geometry import eps_table, material_map
from workloads.pulses import source_values

pytestmark = pytest.mark.gpu


def _cases():
    srr = get_config("cfg1", nx=48, ny=48, t0_steps=200.0, t0_fs=None, fwhm_fs=2.0, n_freq=8,
                     mon_every=2)
    tiny = get_config("cfg0", n_freq=6, mon_every=3)
    return {"tiny": (tiny, 300), "srr_cell": (srr, 400)}


@pytest.mark.parametrize("name", ["tiny", "srr_cell"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fdtd_matches_oracle(name, prec):
    from paper_2209_04487_amd import msqd
    cfg, nsteps = _cases()[name]
    banner(f"fdtd {name} {prec} steps={nsteps}")
    mat = material_map(cfg)
    src = source_values(cfg, 0, nsteps)
    fl = msqd.Fields(msqd.fdtd_desc_from_config(cfg, prec), mat, cfg.freqs)
    for n in range(nsteps):
        fl.step(n, src[n])
    flux = fl.flux().cpu().numpy()
    torch.cuda.synchronize()
    yee = yee_from_config(cfg, mat, eps_table(cfg))
    mon = FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k, cfg.freqs, cfg.dt, cfg.mon_every)
    for n in range(nsteps):
        yee.update_H()
        yee.update_E(src[n], cfg.src_k)
        mon.sample(yee, n)
    tol = 1e-11 if prec == "fp64" else 2e-4
    emax = max(np.abs(e).max() for e in yee.E)
    hmax = max(np.abs(h).max() for h in yee.H)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(fl, nm).cpu().numpy() - yee.E[c]).max() < tol * emax, nm
    for c, nm in enumerate(["Hx", "Hy", "Hz"]):
        assert np.abs(getattr(fl, nm).cpu().numpy() - yee.H[c]).max() < tol * hmax, nm
    for c, nm in enumerate(["JDx", "JDy", "JDz"]):
        ref = yee.JD[c]
        if np.abs(ref).max() > 0:
            assert rel_err(getattr(fl, nm).cpu().numpy(), ref) < 10 * tol, nm
    # CPML auxiliaries: planes k < npml then k >= nz - npml
    npml = cfg.npml
    psi = fl.psi.cpu().numpy()[: 4 * 2 * npml * cfg.ny * cfg.nx].reshape(4, 2 * npml, cfg.ny, cfg.nx)
    for q, ref in enumerate([yee.psi_Ex, yee.psi_Ey, yee.psi_Hx, yee.psi_Hy]):
        refp = np.concatenate([ref[:npml], ref[cfg.nz - npml:]])
        scale = max(np.abs(refp).max(), 1e-300)
        assert np.abs(psi[q] - refp).max() < 10 * tol * scale, q
    dft = fl.dft_planes().cpu().numpy()
    for c, ref in enumerate([mon.Ex, mon.Ey, mon.Hx, mon.Hy]):
        assert rel_err(dft[c], ref) < 10 * tol, c
    assert rel_err(flux, mon.flux()) < 100 * tol
