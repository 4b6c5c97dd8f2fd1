"""GPU parity of the (j, m)-basis molecular step (all three field components)
with the FP64 oracle: the step element by element on seeded random states and
fields (FP64 1e-11, FP32 3e-5 of the largest amplitude), the dipole vector,
norm and yield readouts, and the coupled step on the tiny workload with the
pulse polarised along x (FP64, 1e-10 on the three-component dipole trace, all
field components and the cell polarisation).  j_max = 1 runs the closed-form
kernel, 2 <= j_max <= 5 the general one (rotation to the field frame and the
per-m' transforms of cos(theta)); the oracle diagonalises A(E) directly."""

import numpy as np
import pytest
import torch

from gpu_helpers import TOL, banner, random_state, rel_err
from oracle.coupled import CoupledOracle
from oracle.molecule_jm import jm_model_from_config
from workloads import get_config
from workloads.molecule_inputs import potentials
from workloads.pulses import source_values

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,n_r,n_mol,n_steps", [("fp64", 128, 7, 3), ("fp64", 256, 3, 2),
                                                    ("fp64", 64, 2, 4), ("fp32", 256, 5, 2),
                                                    ("mixed", 128, 9, 3), ("fp32", 256, 5, 1),
                                                    ("mixed", 128, 9, 1)])
def test_jm_step_matches_oracle(prec, n_r, n_mol, n_steps):
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0", n_r=n_r, j_max=1, basis="jm", n_mol=n_mol)
    banner(f"jm qd_step {prec} n_r={n_r} n_mol={n_mol} steps={n_steps}")
    mols = msqd.Molecules.from_config(cfg, prec=prec)
    dr = (cfg.r_max - cfg.r_min) / n_r
    psi = random_state(n_r + n_mol, n_mol, 4, n_r, dr)
    mols.psi.copy_(torch.as_tensor(psi).to(mols.psi.dtype))
    rng = np.random.default_rng(n_mol)
    E3 = rng.uniform(-0.05, 0.05, (n_mol, 3))
    E3[0] = 0.0                               # a molecule with no field at all
    E3[1] = [1e-30, 0.0, 0.0]                 # a vanishing field (series branch, no division)
    if n_mol > 2:
        E3[2] = [0.3, -0.2, 0.25]             # a strong field (large-angle branch in every form)
    mols.step(torch.as_tensor(E3, device="cuda"), n_steps=n_steps)
    d, nrm, yld = mols.readout()
    torch.cuda.synchronize()
    ug, ue, mu = potentials(cfg)
    om = jm_model_from_config(cfg, ug, ue, mu)
    p = psi.copy() if prec == "fp64" else psi.astype(np.complex64).astype(np.complex128)
    ab = np.zeros(n_mol)
    for _ in range(n_steps):
        p, ab = om.step(p, E3, ab)
    tol = TOL[prec]
    assert rel_err(mols.psi.to(torch.complex128).cpu().numpy(), p) < tol
    assert rel_err(mols.d.cpu().numpy(), om.dipole(p)) < 10 * tol
    assert rel_err(d.cpu().numpy(), om.dipole(p)) < 10 * tol
    np.testing.assert_allclose(nrm.cpu().numpy(), om.norm(p), rtol=10 * tol)
    np.testing.assert_allclose(mols.absorbed.cpu().numpy(), ab, rtol=10 * tol, atol=1e-12)


@pytest.mark.parametrize("prec,n_r,j_max,n_mol,n_steps", [("fp64", 128, 2, 7, 3), ("fp64", 64, 5, 6, 2),
                                                          ("fp64", 256, 3, 5, 2), ("fp64", 64, 4, 6, 1),
                                                          ("fp32", 256, 5, 6, 1), ("fp32", 256, 5, 6, 2),
                                                          ("fp32", 256, 2, 6, 1), ("mixed", 128, 4, 6, 1),
                                                          ("fp32", 512, 3, 6, 1), ("fp32", 64, 3, 6, 3),
                                                          ("fp64", 512, 2, 5, 1), ("fp32", 512, 4, 5, 1)])
def test_jm_general_step_matches_oracle(prec, n_r, j_max, n_mol, n_steps):
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0", n_r=n_r, j_max=j_max, basis="jm", n_mol=n_mol)
    nb = (j_max + 1) ** 2
    banner(f"jm general qd_step {prec} n_r={n_r} j_max={j_max} n_mol={n_mol} steps={n_steps}")
    mols = msqd.Molecules.from_config(cfg, prec=prec)
    dr = (cfg.r_max - cfg.r_min) / n_r
    psi = random_state(1000 + 31 * j_max + n_r, n_mol, nb, n_r, dr)
    mols.psi.copy_(torch.as_tensor(psi).to(mols.psi.dtype))
    rng = np.random.default_rng(n_mol + j_max)
    E3 = rng.uniform(-0.05, 0.05, (n_mol, 3))
    E3[0] = 0.0                               # no field: the rotation is the identity
    E3[1] = [0.0, 0.0, -0.04]                 # along -z: beta = pi, alpha undefined
    E3[2] = [0.3, -0.2, 0.25]                 # a strong field (large-angle branch)
    E3[3] = [0.0, 0.0, 0.03]                  # along +z: beta = 0
    E3[4] = [1e-30, 0.0, 0.0]                 # a vanishing field
    mols.step(torch.as_tensor(E3, device="cuda"), n_steps=n_steps)
    d, nrm, yld = mols.readout()
    torch.cuda.synchronize()
    ug, ue, mu = potentials(cfg)
    om = jm_model_from_config(cfg, ug, ue, mu)
    p = psi.copy() if prec == "fp64" else psi.astype(np.complex64).astype(np.complex128)
    ab = np.zeros(n_mol)
    for _ in range(n_steps):
        p, ab = om.step(p, E3, ab)
    tol = TOL[prec]
    assert rel_err(mols.psi.to(torch.complex128).cpu().numpy(), p) < tol
    assert rel_err(mols.d.cpu().numpy(), om.dipole(p)) < 10 * tol
    assert rel_err(d.cpu().numpy(), om.dipole(p)) < 10 * tol
    np.testing.assert_allclose(nrm.cpu().numpy(), om.norm(p), rtol=10 * tol)
    np.testing.assert_allclose(yld.cpu().numpy(), om.dissociated(p, ab), rtol=10 * tol, atol=1e-12)
    np.testing.assert_allclose(mols.absorbed.cpu().numpy(), ab, rtol=10 * tol, atol=1e-12)


def test_jm_general_coupled_tiny_fp64_matches_oracle():
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0", j_max=2, basis="jm", mol_weight=3e3)
    nsteps = 120
    banner(f"jm general coupled cfg0 fp64 j_max=2 {nsteps} steps")
    src = source_values(cfg, 0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64")
    D = np.zeros((nsteps, 3))
    for n in range(nsteps):
        sysm.step(src[n:n + 1])
        D[n] = sysm.mol.d.sum(dim=0).cpu().numpy()
    o = CoupledOracle(cfg)
    tr = o.run(src)
    assert np.abs(tr["D"][:, 0]).max() > 0
    assert np.linalg.norm(D - tr["D"]) / np.linalg.norm(tr["D"]) < 1e-10
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    assert rel_err(sysm.P_c.cpu().numpy(), o.P.T) < 1e-10


def test_jm_general_multirate_fp64_matches_oracle():
    """Multi-rate coupling with the general (j, m) basis: j_max = 2, one
    molecular step of 4 dt every 4 field steps, the three-component current
    held in between; steps 150..330 of the tiny workload, FP64, 1e-10."""
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0", j_max=2, basis="jm", mol_weight=3e3)
    n0, nsteps, M, chunk = 150, 180, 4, 3
    banner(f"jm general coupled cfg0 fp64 j_max=2 multi-rate M={M}, steps {n0}..{n0 + nsteps}")
    src = source_values(cfg, n0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64", mol_every=M)
    sysm.n = n0
    D = np.zeros((nsteps, 3))
    for s in range(0, nsteps, chunk):
        sysm.step(src[s:s + chunk])
        D[s:s + chunk] = sysm.mol.d.sum(dim=0).cpu().numpy()
    o = CoupledOracle(cfg, mol_every=M)
    Do = np.zeros((nsteps, 3))
    for s in range(nsteps):
        o.step(n0 + s, src[s])
        Do[s] = o.d.sum(axis=0)
    idx = np.arange(chunk - 1, nsteps, chunk)
    assert np.abs(Do[idx]).max() > 0
    assert np.linalg.norm(D[idx] - Do[idx]) / np.linalg.norm(Do[idx]) < 1e-10
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    assert rel_err(sysm.P_c.cpu().numpy(), o.P.T) < 1e-10


def test_jm_coupled_tiny_fp64_matches_oracle():
    from paper_2209_04487_amd import msqd
    cfg = get_config("cfg0", j_max=1, basis="jm", mol_weight=3e3)
    nsteps = 300
    banner(f"jm coupled cfg0 fp64 {nsteps} steps")
    src = source_values(cfg, 0, nsteps)
    sysm = msqd.Coupled(cfg, prec="fp64")
    D = np.zeros((nsteps, 3))
    for n in range(nsteps):
        sysm.step(src[n:n + 1])
        D[n] = sysm.mol.d.sum(dim=0).cpu().numpy()
    o = CoupledOracle(cfg)
    tr = o.run(src)
    assert np.abs(tr["D"][:, 0]).max() > 0
    assert np.linalg.norm(D - tr["D"]) / np.linalg.norm(tr["D"]) < 1e-10
    f = sysm.fields
    emax = max(np.abs(e).max() for e in o.yee.E)
    for c, nm in enumerate(["Ex", "Ey", "Ez"]):
        assert np.abs(getattr(f, nm).cpu().numpy() - o.yee.E[c]).max() < 1e-10 * emax, nm
    assert rel_err(sysm.mol.psi.cpu().numpy(), o.psi) < 1e-10
    assert rel_err(sysm.P_c.cpu().numpy(), o.P.T) < 1e-10
    assert rel_err(sysm.E_mol.cpu().numpy(), tr["E_mol"][-1]) < 1e-10
