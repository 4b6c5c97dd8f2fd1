"""Oracle: the self-consistent Maxwell-Schroedinger step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Efficient numerical implementation ...": each molecule is driven by
the local electric field; its induced dipole, multiplied by the molecular
number density (mean-field approximation), gives the macroscopic
polarisation P, and J = dP/dt enters Ampere's law (Eq. (1)).

One coupled step n -> n+1, in this order:
  1. H^{n+1/2} from E^n                                      (Eq. (1))
  2. E_mol,i = E_x^n at the molecule's E_x edge, in atomic units
  3. every molecule: psi^n -> psi^{n+1} under E_mol,i held over the step
  4. d_i^{n+1}; P_c^{n+1} = (w / dx^3) sum_{i in c} d_i (e a0), summed cell by
     cell in molecule-index order; J_mol,c = (P_c^{n+1} - P_c^n) / dt
  5. E^{n+1} with the Drude, molecular and source currents    (Eqs. (1), (2))
  6. flux-monitor sample

Multi-rate coupling (the paper advances its molecules only every 40th field
step, section on molecular mapping): with mol_every = M the molecules take
one step of M dt at every field step n with n % M == 0, driven by E_x^n held
over the M field steps; P jumps to its new value there and the current
J_mol = (P_new - P_old) / (M dt) is applied, unchanged, at each of the M field
steps that follow (P linear in time between molecular updates).  M = 1 is the
scheme above.
"""

from __future__ import annotations

import numpy as np

from workloads.geometry import eps_table, material_map
from workloads.molecule_inputs import morse_v0, potentials

from .fdtd import FluxMonitor, yee_from_config
from .maps import cells_from_config, csr
from .molecule import model_from_config
from .molecule_jm import jm_model_from_config

E_AU = 5.14220674763e11      # V/m
EA0 = 8.4783536255e-30       # C m


class CoupledOracle:
    def __init__(self, cfg, n_mol=None, cells=None, mat=None, yee=None, mol_every=1):
        self.cfg = cfg
        self.mol_every = int(mol_every)
        if mat is None:
            mat = material_map(cfg)
        self.mat = mat
        self.yee = yee if yee is not None else yee_from_config(cfg, mat, eps_table(cfg))
        ug, ue, mu = potentials(cfg)
        # rotational basis: m = 0 J lines with the field along the axis, or
        # all (j, m) with the three field components at each cell's own edges
        self.jm = getattr(cfg, "basis", "m0") == "jm"
        make = jm_model_from_config if self.jm else model_from_config
        self.mol = make(cfg, ug, ue, mu, dt_au=cfg.dt_au * self.mol_every)
        if cells is None:
            cells = cells_from_config(cfg)
        if n_mol is not None:
            cells = cells[:n_mol]
        self.cells = np.asarray(cells, dtype=np.int64)
        self.n_mol = len(self.cells)
        self.occ, self.ptr, self.perm = csr(self.cells)
        self.psi = self.mol.initial_state(self.n_mol, morse_v0(cfg))
        self.absorbed = np.zeros(self.n_mol)
        nc = 3 if self.jm else 1
        self.P = np.zeros((nc, len(self.occ))) if self.jm else np.zeros(len(self.occ))
        self.Jmol = np.zeros_like(self.P)
        self.monitor = FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k, cfg.freqs, cfg.dt, cfg.mon_every)
        self.monitor2 = (FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k2, cfg.freqs, cfg.dt, cfg.mon_every)
                         if cfg.mon_k2 else None)
        self.d = np.zeros((self.n_mol, 3)) if self.jm else np.zeros(self.n_mol)
        self.e_mol = np.zeros((self.n_mol, 3)) if self.jm else np.zeros(self.n_mol)

    def cell_sums(self, d):
        """Per occupied cell, the sum of its molecules' dipoles in CSR order."""
        out = np.zeros(len(self.occ))
        for c in range(len(self.occ)):
            acc = 0.0
            for idx in range(self.ptr[c], self.ptr[c + 1]):
                acc += d[self.perm[idx]]
            out[c] = acc
        return out

    def step(self, n, src_value):
        """Field step n -> n+1; the molecules advance when n % mol_every == 0.
        Returns the field the molecules saw at their last update."""
        cfg = self.cfg
        yee = self.yee
        yee.update_H()
        if n % self.mol_every == 0:
            if self.jm:
                e_mol = np.stack([yee.E[c].reshape(-1)[self.cells] for c in range(3)], axis=1) / E_AU
            else:
                e_mol = yee.E[0].reshape(-1)[self.cells] / E_AU
            self.psi, self.absorbed = self.mol.step(self.psi, e_mol, self.absorbed)
            self.d = self.mol.dipole(self.psi)
            if self.jm:
                sums = np.stack([self.cell_sums(self.d[:, c]) for c in range(3)])
            else:
                sums = self.cell_sums(self.d)
            P_new = cfg.mol_weight * sums * EA0 / cfg.dx ** 3
            self.Jmol = (P_new - self.P) / (cfg.dt * self.mol_every)
            self.P = P_new
            self.e_mol = e_mol
        yee.update_E(src_value, cfg.src_k, self.occ, self.Jmol)
        self.monitor.sample(yee, n)
        if self.monitor2 is not None:
            self.monitor2.sample(yee, n)
        return self.e_mol

    def run(self, src_values, n0=0, record_fields=False):
        """Run len(src_values) steps from step n0; returns per-step traces."""
        nst = len(src_values)
        shape = self.d.shape
        trace = {"D": np.zeros((nst,) + shape[1:]), "d": np.zeros((nst,) + shape),
                 "E_mol": np.zeros((nst,) + shape)}
        for s in range(nst):
            e_mol = self.step(n0 + s, src_values[s])
            trace["D"][s] = self.d.sum(axis=0)
            trace["d"][s] = self.d
            trace["E_mol"][s] = e_mol
        return trace
