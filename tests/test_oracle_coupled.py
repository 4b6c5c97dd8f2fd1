"""Pins of the oracle's coupling (gather -> molecular step -> P -> J -> E).

- energy balance: in a closed periodic box the field energy lost equals the
  molecular energy gained (Poynting's theorem with J = dP/dt), up to the
  first-order error of holding E^n over the molecular step; this fixes the
  sign of the polarisation current and every unit conversion on the path;
- exact per-cell sums for dyadic-rational dipoles (no rounding at all);
- the tiny workload runs with norm + absorbed = 1 for every molecule;
- multi-rate coupling (molecules every M field steps): the same energy
  balance, first order in the molecular step M dt, and the held current
  J_mol integrates over the field steps to exactly the polarisation change.
"""

from fractions import Fraction

import numpy as np

from oracle.coupled import CoupledOracle
from oracle.fdtd import EPS0, Yee
from workloads import get_config
from workloads.pulses import source_values

EH_J = 4.3597447222071e-18     # hartree in joule


def _h0(mol, psi):
    """<H0> per molecule (hartree): kinetic from the momentum distribution
    plus potential and centrifugal terms."""
    n = mol.n_r
    ph = np.fft.fft(psi, axis=-1)
    kin = np.sum(np.abs(ph) ** 2 * (mol.kappa ** 2 / (2 * mol.mass))[None, None, None, :],
                 axis=(1, 2, 3)) * mol.dr / n
    J = np.arange(mol.n_j)
    V = mol.U[:, None, :] + (J * (J + 1))[None, :, None] / (2 * mol.mass * mol.r[None, None, :] ** 2)
    return kin + np.sum(np.abs(psi) ** 2 * V[None], axis=(1, 2, 3)) * mol.dr


def _closed_box(courant, mol_every=1):
    cfg = get_config("cfg0", nx=2, ny=2, nz=2, courant=courant, mol_weight=1e4,
                     n_mol=8, placement="block", block_lo=0, block_n=2, mon_k=1)
    mat = np.zeros((3, 2, 2, 2), np.uint8)
    yee = Yee(2, 2, 2, cfg.dx, cfg.dt, mat, [1, 1, 1], 0.0, 0.0, 0, periodic_z=True)
    o = CoupledOracle(cfg, mat=mat, yee=yee, mol_every=mol_every)
    yee.E[0][:] = 5e-2 * 5.14220674763e11
    return cfg, o, yee


def test_energy_balance_closed_box():
    imbalance = []
    for courant in (0.5, 0.25):
        cfg, o, yee = _closed_box(courant)
        f0 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
        m0 = cfg.mol_weight * np.sum(_h0(o.mol, o.psi)) * EH_J
        nst = int(round(200 / courant))
        for n in range(nst):
            o.step(n, 0.0)
        f1 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
        m1 = cfg.mol_weight * np.sum(_h0(o.mol, o.psi)) * EH_J
        assert f1 < f0 and m1 > m0           # energy flows from field to molecules
        imbalance.append(((f1 + m1) - (f0 + m0)) / (m1 - m0))
    assert abs(imbalance[0]) < 0.25
    assert 1.6 < imbalance[0] / imbalance[1] < 2.4, imbalance   # first order in dt


def test_cell_sums_exact_for_dyadic_dipoles():
    cfg = get_config("cfg0", nx=8, ny=8, nz=24, placement="slab", slab_k0=10, slab_nk=2,
                     n_mol=300, seed=9)
    o = CoupledOracle(cfg)
    rng = np.random.default_rng(0)
    d = rng.integers(-2 ** 20, 2 ** 20, size=o.n_mol) / 2.0 ** 12
    sums = o.cell_sums(d)
    for c, cell in enumerate(o.occ):
        exact = sum(Fraction(float(d[i])) for i in range(o.n_mol) if o.cells[i] == cell)
        assert Fraction(float(sums[c])) == exact
    assert o.ptr[-1] == o.n_mol


def test_tiny_workload_conserves_probability():
    cfg = get_config("cfg0")
    o = CoupledOracle(cfg)
    o.run(source_values(cfg, 0, 60))
    np.testing.assert_allclose(o.mol.norm(o.psi) + o.absorbed, 1.0, atol=1e-13)


def _imbalance(courant, mol_every, t_units=200):
    cfg, o, yee = _closed_box(courant, mol_every)
    f0 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
    m0 = cfg.mol_weight * np.sum(_h0(o.mol, o.psi)) * EH_J
    nst = int(round(t_units / courant))
    nst -= nst % mol_every
    for n in range(nst):
        o.step(n, 0.0)
    f1 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
    m1 = cfg.mol_weight * np.sum(_h0(o.mol, o.psi)) * EH_J
    assert f1 < f0 and m1 > m0
    return ((f1 + m1) - (f0 + m0)) / (m1 - m0)


def test_multirate_energy_balance_first_order_in_molecular_step():
    """Molecules every M field steps (M dt per molecular step): the balance
    error scales with M dt.  A current that is not divided by M, or applied
    at only one of the M field steps, breaks the balance at zeroth order."""
    i2 = _imbalance(0.25, 2)
    i4 = _imbalance(0.25, 4)
    i1_half = _imbalance(0.5, 1)
    assert abs(i4) < 0.5
    assert 1.6 < i4 / i2 < 2.4, (i2, i4)
    # the same molecular step (M dt = 0.5 dx/c) on a finer field grid: close
    assert abs(i2 - i1_half) < 0.1 * abs(i1_half), (i2, i1_half)


def test_multirate_current_integrates_to_polarisation():
    cfg = get_config("cfg0", n_mol=64)
    o = CoupledOracle(cfg, mol_every=5)
    src = source_values(cfg, 200, 40)
    acc = np.zeros(len(o.occ))
    P0 = o.P.copy()
    for s_, v in enumerate(src):
        o.step(200 + s_, v)
        acc += o.Jmol * cfg.dt
    # 40 field steps = 8 molecular updates, the last at step 235
    np.testing.assert_allclose(acc, o.P - P0, rtol=1e-12, atol=1e-12 * np.abs(o.P).max())
    assert np.abs(o.P).max() > 0
