"""GPU parity of the whole coupled step (coupled_step) with the FP64 oracle on
the tiny workload (24^3 grid, 64 molecules, 500 steps): the ensemble dipole
trace D(t) = sum_i d_i(t), every molecule's dipole at every step, the final
fields, wavepackets, absorbed norms, cell polarisation and monitor flux.

FP64 form: 1e-10 relative (the spec parity bar).  FP32 / mixed forms:
the dipole trace within 1e-4 relative L2 of the FP64 oracle."""

import numpy as np
import pytest
import torch

from gpu_helpers import banner, rel_err
from oracle.coupled import CoupledOracle
from workloads import get_config
from workloads.pulses import source_values

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _oracle(cfg, nsteps):
    key = (cfg.name, nsteps)
    if key not in _ORACLE:
        o = CoupledOracle(cfg)
        tr = o.run(source_values(cfg, 0, nsteps))
        _ORACLE[key] = (o, tr)
    return _ORACLE[key]


def _gpu_run(cfg, prec, nsteps):
    """Per-step dipoles of every molecule and the library's ensemble sums
    (dipole_readout: sum d, sum norm, sum yield) after every step."""
    from paper_2209_04487_amd import msqd
    sysm = msqd.Coupled(cfg, prec=prec)
    src = source_values(cfg, 0, nsteps)
    d = np.zeros((nsteps, sysm.mol.desc.n_mol))
    sums = torch.zeros((nsteps, sysm.mol.n_sums), dtype=torch.float64, device="cuda")
    for n in range(nsteps):
        sysm.step(src[n:n + 1])
        d[n] = sysm.mol.d.cpu().numpy()
        sysm.ensemble_sums(sums[n])
    torch.cuda.synchronize()
    return sysm, d, sums.cpu().numpy()


def test_coupled_tiny_fp64_matches_oracle():
    cfg = get_config("cfg0")
    nsteps = cfg.n_steps
    banner(f"coupled cfg0 fp64 {nsteps} steps")
    sysm, d, sums = _gpu_run(cfg, "fp64", nsteps)
    o, tr = _oracle(cfg, nsteps)
    D = sums[:, 0]
    assert np.linalg.norm(D - tr["D"]) / np.linalg.norm(tr["D"]) < 1e-10
    assert rel_err(d, tr["d"]) < 1e-10
    # the ensemble sums equal the sums of the per-molecule values (the
    # coupled step's own dipoles), and the final norm and yield sums the oracle's
    np.testing.assert_allclose(D, d.sum(axis=1), rtol=1e-13, atol=1e-13 * np.abs(D).max())
    np.testing.assert_allclose(sums[-1, 1], o.mol.norm(o.psi).sum(), rtol=1e-12)
    np.testing.assert_allclose(sums[-1, 2], o.mol.dissociated(o.psi, o.absorbed).sum(), rtol=1e-10,
                               atol=1e-20)
    # fields: relative to the field scale (the scattered E_y, E_z are small
    # differences of nearly equal cell currents, so their own scale is not a
    # meaningful denominator)
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    hmax = max(np.abs(h).max() for h in o.yee.H)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    for c, nm in enumerate(["Hx", "Hy", "Hz"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.H[c]).max() < 1e-10 * hmax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    np.testing.assert_allclose(sysm.mol.absorbed.cpu().numpy(), o.absorbed, rtol=1e-10)
    assert rel_err(sysm.P_c.cpu().numpy(), o.P) < 1e-10
    assert rel_err(sysm.E_mol.cpu().numpy(), tr["E_mol"][-1]) < 1e-10
    assert rel_err(f.flux().cpu().numpy(), o.monitor.flux()) < 1e-9
    dd, nn, yy = sysm.mol.readout()
    np.testing.assert_allclose(nn.cpu().numpy() + sysm.mol.absorbed.cpu().numpy(), 1.0, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_coupled_tiny_reduced_precision_dipole_error(prec):
    cfg = get_config("cfg0")
    nsteps = cfg.n_steps
    banner(f"coupled cfg0 {prec} {nsteps} steps")
    sysm, d, sums = _gpu_run(cfg, prec, nsteps)
    o, tr = _oracle(cfg, nsteps)
    D = sums[:, 0]
    err = np.linalg.norm(D - tr["D"]) / np.linalg.norm(tr["D"])
    print(f"{prec} relative dipole-trace error {err:.3e}")
    assert err < 1e-4


@pytest.mark.parametrize("mol_every", [4, 7])
def test_coupled_multirate_fp64_matches_oracle(mol_every):
    """Molecules every M field steps (one molecular step of M dt under E_x^n,
    the held current applied at every field step): the tiny workload over
    steps 150..400 (the pulse crosses the molecules), FP64, against the
    oracle's multi-rate scheme at 1e-10.  M = 7 does not divide the window
    start or length, so updates fall inside calls of several steps."""
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0")
    n0, nsteps = 150, 250
    banner(f"coupled cfg0 fp64 multi-rate M={mol_every}, steps {n0}..{n0 + nsteps}")
    src = source_values(cfg, n0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64", mol_every=mol_every)
    sysm.n = n0
    D = np.zeros(nsteps)
    chunk = 3
    for s in range(0, nsteps, chunk):
        sysm.step(src[s:s + chunk])
        D[s:s + chunk] = float(sysm.ensemble_sums()[0])   # constant between updates
    torch.cuda.synchronize()
    o = CoupledOracle(cfg, mol_every=mol_every)
    Do = np.zeros(nsteps)
    for s in range(nsteps):
        o.step(n0 + s, src[s])
        Do[s] = o.d.sum()
    idx = np.arange(chunk - 1, nsteps, chunk)
    assert np.abs(Do[idx]).max() > 0
    assert np.linalg.norm(D[idx] - Do[idx]) / np.linalg.norm(Do[idx]) < 1e-10
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    assert rel_err(sysm.P_c.cpu().numpy(), o.P) < 1e-10
    assert rel_err(sysm.J_mol.cpu().numpy(), o.Jmol) < 1e-10


def test_coupled_multirate_rejects_step_mismatch():
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0")
    sysm = msqd.Coupled(cfg, prec="fp64", mol_every=4)
    sysm.desc.mol_every = 5            # molecules were built for 4 dt
    with pytest.raises(msqd.MsqdError):
        sysm.step(np.zeros(2))


def _state_tensors(sysm):
    t = {k: sysm.fields.t[k] for k in ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "JDx", "JDy", "JDz", "psi", "dft"]}
    t.update(mol_psi=sysm.mol.psi, absorbed=sysm.mol.absorbed, d=sysm.mol.d, P_c=sysm.P_c, J_mol=sysm.J_mol,
             E_mol=sysm.E_mol)
    return t


@pytest.mark.parametrize("basis,prec,mol_every", [("m0", "mixed", 1), ("m0", "mixed", 5), ("m0", "fp32", 5),
                                                   ("m0", "fp64", 5), ("jm", "fp64", 3)])
def test_held_current_path_is_bit_identical(basis, prec, mol_every):
    """coupled_step with the held-current array (the E update subtracts the
    molecular current) against the separate pass after the E update: every
    field, wavepacket, absorbed norm, dipole and polarisation array bit for bit,
    over calls of uneven length that start on and between molecular updates,
    and after a restore between updates (the call rebuilds the held array)."""
    from paper_2209_04487_amd import msqd
    over = dict(j_max=1, basis="jm", mol_weight=3e3) if basis == "jm" else {}
    cfg = get_config("cfg0", **over)
    n0, nsteps = 150, 60
    banner(f"held current {basis} {prec} M={mol_every}, steps {n0}..{n0 + nsteps}")
    src = source_values(cfg, n0, nsteps)
    runs = []
    for held in (True, False):
        sysm = msqd.Coupled(cfg, prec=prec, mol_every=mol_every, held=held)
        assert (sysm.E_held is not None) == held
        sysm.n = n0
        s, snap = 0, None
        for chunk in [3, 1, 7, 2, 11, 4, 9, 6]:
            sysm.step(src[s:s + chunk])
            s += chunk
            if s == 13:
                snap = sysm.snapshot()
        sysm.restore(snap)                 # back to step n0 + 13
        sysm.step(src[13:13 + 8])
        sysm.step(src[21:21 + 5])
        torch.cuda.synchronize()
        runs.append({k: v.clone() for k, v in _state_tensors(sysm).items()})
    assert float(runs[0]["J_mol"].abs().max()) > 0
    for k in runs[0]:
        assert torch.equal(runs[0][k], runs[1][k]), k


def test_held_current_outside_its_planes_poisons_the_field():
    """An occupied cell outside the held planes sets its E_x to NaN at the next
    molecular update (cfg0's molecules sit on planes 10..13; plane 23 is given
    as the held range)."""
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0")
    banner("held current outside its planes")
    sysm = msqd.Coupled(cfg, prec="fp64")
    assert (sysm.desc.held_k0, sysm.desc.held_nk) == (10, 4)
    sysm.desc.held_k0, sysm.desc.held_nk = cfg.nz - 1, 1
    sysm.step(source_values(cfg, 0, 1))
    torch.cuda.synchronize()
    ex = sysm.fields.Ex.cpu().numpy().reshape(-1)
    occ = sysm.occ_cell.cpu().numpy()
    assert np.isnan(ex[occ]).all()
    assert np.isfinite(np.delete(ex, occ)).all()
