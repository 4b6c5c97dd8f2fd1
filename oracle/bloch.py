"""Oracle: frozen two-level (Bloch) emitters integrated by the classical
fourth-order Runge-Kutta scheme, and their coupling to the Yee grid.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's comparison workload (section on molecular mapping, the
experiment with frozen ro-vibrational degrees of freedom) replaces each
molecule by a two-level emitter obeying the Bloch equations, advanced by
RK4.  Written here in atomic units for one emitter with transition
frequency w0, transition dipole mu and the interaction -mu E sigma_x (the
field along the dipole):

    H = [[0, V], [V, w0]],  V = -mu E,
    d rho_ee / dt     = 2 V Im(rho_ge) - g1 rho_ee
    d rho_ge / dt     = (i w0 - g2) rho_ge - i V (rho_ee - rho_gg),
    rho_gg = 1 - rho_ee,

with optional population decay g1 and dephasing g2 (zero in the paper's
test).  The dipole is d = mu (rho_ge + rho_eg) = 2 mu Re(rho_ge).  The state
is (rho_ee, Re rho_ge, Im rho_ge); the field E is held over the step, like
the molecular step of the coupled scheme.
"""

from __future__ import annotations

import numpy as np

from workloads.geometry import eps_table, material_map

from .fdtd import FluxMonitor, yee_from_config
from .maps import cells_from_config, csr

E_AU = 5.14220674763e11      # V/m
EA0 = 8.4783536255e-30       # C m


class BlochModel:
    def __init__(self, omega0, mu, dt, gamma1=0.0, gamma2=0.0):
        self.w0 = float(omega0)
        self.mu = float(mu)
        self.dt = float(dt)
        self.g1 = float(gamma1)
        self.g2 = float(gamma2)

    def rhs(self, y, E):
        """Time derivative of y = [rho_ee, Re rho_ge, Im rho_ge] (shape
        [3, n]) under the field E (shape [n], au)."""
        pe, u, v = y
        V = -self.mu * E
        dpe = 2.0 * V * v - self.g1 * pe
        # d(u + i v)/dt = (i w0 - g2)(u + i v) - i V (2 pe - 1)
        du = -self.w0 * v - self.g2 * u
        dv = self.w0 * u - self.g2 * v - V * (2.0 * pe - 1.0)
        return np.array([dpe, du, dv])

    def step(self, y, E):
        """One RK4 step of length dt with E held."""
        h = self.dt
        k1 = self.rhs(y, E)
        k2 = self.rhs(y + 0.5 * h * k1, E)
        k3 = self.rhs(y + 0.5 * h * k2, E)
        k4 = self.rhs(y + h * k3, E)
        return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def dipole(self, y):
        return 2.0 * self.mu * y[1]

    @staticmethod
    def ground(n):
        return np.zeros((3, n))


def bloch_from_config(cfg, dt_au=None):
    """The frozen limit of the workload's molecule: the vertical gap
    U_e(r_e) - U_g(r_e) and the transition dipole mu12(r_e)/sqrt(3) (the
    orientation average of the J = 0 ground state's coupling)."""
    from workloads.molecule_inputs import bloch_parameters
    w0, mu = bloch_parameters(cfg)
    return BlochModel(w0, mu, cfg.dt_au if dt_au is None else dt_au)


class CoupledBlochOracle:
    """The coupled step of the paper's frozen-emitter comparison: the same
    field update, gather, per-cell polarisation and current as the molecular
    scheme, with each emitter advanced by one RK4 step under E_x^n."""

    def __init__(self, cfg, model=None, cells=None, mat=None, yee=None):
        self.cfg = cfg
        if mat is None:
            mat = material_map(cfg)
        self.yee = yee if yee is not None else yee_from_config(cfg, mat, eps_table(cfg))
        self.model = model if model is not None else bloch_from_config(cfg)
        if cells is None:
            cells = cells_from_config(cfg)
        self.cells = np.asarray(cells, dtype=np.int64)
        self.n = len(self.cells)
        self.occ, self.ptr, self.perm = csr(self.cells)
        self.y = BlochModel.ground(self.n)
        self.P = np.zeros(len(self.occ))
        self.Jmol = np.zeros(len(self.occ))
        self.d = np.zeros(self.n)
        self.monitor = FluxMonitor(cfg.ny, cfg.nx, cfg.mon_k, cfg.freqs, cfg.dt, cfg.mon_every)

    def cell_sums(self, d):
        out = np.zeros(len(self.occ))
        for c in range(len(self.occ)):
            acc = 0.0
            for idx in range(self.ptr[c], self.ptr[c + 1]):
                acc += d[self.perm[idx]]
            out[c] = acc
        return out

    def step(self, n, src_value):
        cfg = self.cfg
        yee = self.yee
        yee.update_H()
        e = yee.E[0].reshape(-1)[self.cells] / E_AU
        self.y = self.model.step(self.y, e)
        self.d = self.model.dipole(self.y)
        P_new = cfg.mol_weight * self.cell_sums(self.d) * EA0 / cfg.dx ** 3
        self.Jmol = (P_new - self.P) / cfg.dt
        self.P = P_new
        yee.update_E(src_value, cfg.src_k, self.occ, self.Jmol)
        self.monitor.sample(yee, n)
        return e
