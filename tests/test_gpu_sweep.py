"""GPU parity of the fused field sweep (coupled_step with a spare field set:
H and E of a step in one pass, alternating between two sets of arrays)
against the FP64 oracle.

- field steps alone (no molecules) on the tiny grid (24 x 24: tiles of 32 x 8
  cells ragged in x), a grid ragged in both x and y, one SRR unit cell of the
  silver array (metal, glass, both CPMLs, source, monitor) and the full
  192 x 192 x 120 SRR grid; calls of odd and even lengths, so that the
  alternation ends with a two-kernel step; every E and H component, the
  Drude currents, the CPML auxiliaries and the monitor accumulators.  FP64
  1e-11 of the largest value, FP32 2e-4 (as the two-kernel update);
- the coupled tiny workload (64 molecules, 500 steps) in calls of 10 steps,
  and with multi-rate coupling (M = 4) in calls of 6: wavepackets, dipoles,
  absorbed norms, cell polarisation, fields and flux at 1e-10;
- the precision form of the tiny workload against the two-kernel update of
  the same form (fields to 2e-6 of their peak, the ensemble dipole to 1e-5).
"""

import numpy as np
import pytest
import torch

from gpu_helpers import banner, rel_err
from oracle.coupled import CoupledOracle
from oracle.fdtd import FluxMonitor, yee_from_config
from workloads import get_config
from workloads.geometry import eps_table, material_map
from workloads.pulses import source_values

pytestmark = pytest.mark.gpu

E_NAMES = ["Ex", "Ey", "Ez"]
H_NAMES = ["Hx", "Hy", "Hz"]


def _cases():
    return {
        "tiny": (get_config("cfg0", n_freq=6, mon_every=3), 300),
        "ragged": (get_config("cfg0", nx=40, ny=20, nz=30, n_freq=4, mon_every=2, src_k=8, mon_k=22), 200),
        "srr_cell": (get_config("cfg1", nx=48, ny=48, t0_steps=200.0, t0_fs=None, fwhm_fs=2.0, n_freq=8,
                                mon_every=2), 400),
    }


def _chunks(nsteps):
    """Call lengths mixing odd and even counts."""
    out, seq, i = [], [7, 10, 1, 2, 33, 16], 0
    while sum(out) < nsteps:
        out.append(min(seq[i % len(seq)], nsteps - sum(out)))
        i += 1
    return out


def _field_run(cfg, prec, nsteps):
    from paper_2209_04487_amd import msqd
    mat = material_map(cfg)
    src = source_values(cfg, 0, nsteps)
    sysm = msqd.Coupled(cfg, prec=prec, cells=np.zeros(0, np.int32), mat=mat)
    assert sysm.fields.f.spare is not None
    for c in _chunks(nsteps):
        sysm.step(src[sysm.n:sysm.n + c])
    torch.cuda.synchronize()
    yee = yee_from_config(cfg, mat, eps_table(cfg))
    mon = FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k, cfg.freqs, cfg.dt, cfg.mon_every)
    for n in range(nsteps):
        yee.update_H()
        yee.update_E(src[n], cfg.src_k)
        mon.sample(yee, n)
    return sysm.fields, yee, mon


def _compare_fields(fl, yee, cfg, tol):
    emax = max(np.abs(e).max() for e in yee.E)
    hmax = max(np.abs(h).max() for h in yee.H)
    for c, nm in enumerate(E_NAMES):
        assert np.abs(getattr(fl, nm).cpu().numpy() - yee.E[c]).max() < tol * emax, nm
    for c, nm in enumerate(H_NAMES):
        assert np.abs(getattr(fl, nm).cpu().numpy() - yee.H[c]).max() < tol * hmax, nm
    for c, nm in enumerate(["JDx", "JDy", "JDz"]):
        ref = yee.JD[c]
        if np.abs(ref).max() > 0:
            assert rel_err(getattr(fl, nm).cpu().numpy(), ref) < 10 * tol, nm
    npml = cfg.npml
    psi = fl.psi.cpu().numpy()[: 4 * 2 * npml * cfg.ny * cfg.nx].reshape(4, 2 * npml, cfg.ny, cfg.nx)
    for q, ref in enumerate([yee.psi_Ex, yee.psi_Ey, yee.psi_Hx, yee.psi_Hy]):
        refp = np.concatenate([ref[:npml], ref[cfg.nz - npml:]])
        scale = max(np.abs(refp).max(), 1e-300)
        assert np.abs(psi[q] - refp).max() < 10 * tol * scale, q


@pytest.mark.parametrize("name", ["tiny", "ragged", "srr_cell"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_field_steps_match_oracle(name, prec):
    cfg, nsteps = _cases()[name]
    banner(f"fused sweep {name} {prec}: {cfg.nx}x{cfg.ny}x{cfg.nz}, {nsteps} steps in calls {_chunks(nsteps)}")
    fl, yee, mon = _field_run(cfg, prec, nsteps)
    tol = 1e-11 if prec == "fp64" else 2e-4
    _compare_fields(fl, yee, cfg, tol)
    dft = fl.dft_planes().cpu().numpy()
    for c, ref in enumerate([mon.Ex, mon.Ey, mon.Hx, mon.Hy]):
        assert rel_err(dft[c], ref) < 10 * tol, c


def test_fused_full_grid_fp64():
    """The full SRR grid, the pulse across the rings, the slab and the lower
    CPML (240 steps in calls of 40, 80 and 120), and the monitor as the
    benchmark runs it (32 frequencies every 4 steps)."""
    cfg = get_config("cfg1", t0_steps=30.0, t0_fs=None, fwhm_fs=1.0)
    nsteps = 240
    banner(f"fused sweep full grid cfg1 fp64: {cfg.nx}x{cfg.ny}x{cfg.nz}, {nsteps} steps")
    from paper_2209_04487_amd import msqd
    mat = material_map(cfg)
    src = source_values(cfg, 0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64", cells=np.zeros(0, np.int32), mat=mat)
    for c in (40, 80, 120):
        sysm.step(src[sysm.n:sysm.n + c])
    torch.cuda.synchronize()
    yee = yee_from_config(cfg, mat, eps_table(cfg))
    mon = FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k, cfg.freqs, cfg.dt, cfg.mon_every)
    for n in range(nsteps):
        yee.update_H()
        yee.update_E(src[n], cfg.src_k)
        mon.sample(yee, n)
    _compare_fields(sysm.fields, yee, cfg, 1e-11)
    dft = sysm.fields.dft_planes().cpu().numpy()
    for c, ref in enumerate([mon.Ex, mon.Ey, mon.Hx, mon.Hy]):
        assert np.abs(ref).max() > 0
        assert rel_err(dft[c], ref) < 1e-10, c
    assert rel_err(sysm.fields.flux().cpu().numpy(), mon.flux()) < 1e-9


@pytest.mark.parametrize("mol_every,chunk", [(1, 10), (4, 6)])
def test_fused_coupled_tiny_fp64_matches_oracle(mol_every, chunk):
    """The coupled tiny workload with the fused sweep: the molecules gather
    E^n from whichever set holds step n, the polarisation current lands on
    the set the sweep wrote."""
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0")
    nsteps = 500 if mol_every == 1 else 250
    banner(f"fused sweep coupled cfg0 fp64 M={mol_every}, {nsteps} steps in calls of {chunk}")
    src = source_values(cfg, 0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64", mol_every=mol_every)
    D = []
    while sysm.n < nsteps:
        c = min(chunk, nsteps - sysm.n)
        sysm.step(src[sysm.n:sysm.n + c])
        D.append(float(sysm.ensemble_sums()[0]))
    torch.cuda.synchronize()
    o = CoupledOracle(cfg, mol_every=mol_every)
    Do = []
    for n in range(nsteps):
        o.step(n, src[n])
        if (n + 1) % chunk == 0 or n + 1 == nsteps:
            Do.append(o.d.sum())
    D, Do = np.array(D), np.array(Do)
    assert np.abs(Do).max() > 0
    assert np.linalg.norm(D - Do) / np.linalg.norm(Do) < 1e-10
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    hmax = max(np.abs(h).max() for h in o.yee.H)
    for c, nm in enumerate(E_NAMES):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    for c, nm in enumerate(H_NAMES):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.H[c]).max() < 1e-10 * hmax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    assert rel_err(sysm.P_c.cpu().numpy(), o.P) < 1e-10
    # the absorbed norms here are FP64 round-off of the far Morse tail (about 6e-13)
    np.testing.assert_allclose(sysm.mol.absorbed.cpu().numpy(), o.absorbed, rtol=1e-10, atol=1e-20)
    assert rel_err(f.flux().cpu().numpy(), o.monitor.flux()) < 1e-9


def test_fused_mixed_form_against_two_kernel_update():
    """The precision form of the tiny workload, 200 steps: the fused sweep
    (one call) against the two-kernel update (one step per call) of the same
    form; they differ only by FP32 rounding order."""
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0")
    nsteps = 200
    banner("fused sweep vs two-kernel update, cfg0 mixed")
    src = source_values(cfg, 0, nsteps)
    a = msqd.Coupled(cfg, prec="mixed")
    a.step(src)
    b = msqd.Coupled(cfg, prec="mixed")
    for n in range(nsteps):
        b.step(src[n:n + 1])
    torch.cuda.synchronize()
    for nm in E_NAMES + H_NAMES:
        x, y = getattr(a.fields, nm).double(), getattr(b.fields, nm).double()
        assert float((x - y).abs().max()) <= 2e-6 * float(y.abs().max()), nm
    da, db = float(a.ensemble_sums()[0]), float(b.ensemble_sums()[0])
    assert abs(da - db) <= 1e-5 * abs(db)
