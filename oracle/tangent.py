"""Oracle: forward-mode (tangent-linear) derivative of the coupled run.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The reference for the hand-written adjoint.  The differentiated run is the
coupled step of Eqs. (1)-(5) as in oracle.coupled; the objective is the
dissociated population studied in the paper's application section on
collective dissociation near plasmonic interfaces, at the end of the run, Y = mean_i [sum_{r > r_diss} |psi_i|^2 dr + absorbed_i],
and its derivative along a direction of the incident-field samples,
dY = sum_n (dY/dsrc[n]) dsrc[n], propagated forward alongside the state.

Every factor of the step is linear in the state except the dipole rotation,
whose angle depends on the gathered field; the tangent of each factor is the
factor itself applied to the tangent state, plus, for the rotation,
dPhi' = R(phi) dPhi + (d phi) (i sigma_x) R(phi) Phi with d phi = mu12 x_k dt dE.
The field solver is linear, so the tangent fields obey the same update with
the tangent source and the tangent polarisation current.
"""

from __future__ import annotations

import numpy as np

from .coupled import E_AU, EA0, CoupledOracle
from .fdtd import yee_from_config


class CoupledTangent:
    def __init__(self, cfg, **kw):
        self.base = CoupledOracle(cfg, **kw)
        b = self.base
        from workloads.geometry import eps_table
        self.dyee = yee_from_config(cfg, b.mat, eps_table(cfg))
        self.dpsi = np.zeros_like(b.psi)
        self.dab = np.zeros(b.n_mol)
        self.dP = np.zeros(len(b.occ))

    def _mol_step(self, E, dE):
        m = self.base.mol
        psi, dpsi = self.base.psi, self.dpsi
        psi, dpsi = m.kinetic_half(psi), m.kinetic_half(dpsi)
        psi, dpsi = m.potential_half(psi), m.potential_half(dpsi)
        # rotation on the angular grid with its field derivative
        phi = m.rotation_angle(E)
        dphi = m.rotation_angle(dE)
        c, s = np.cos(phi), np.sin(phi)
        P, dP = m.to_angle(psi), m.to_angle(dpsi)
        g, e, dg, de = P[:, 0], P[:, 1], dP[:, 0], dP[:, 1]
        g2 = c * g + 1j * s * e
        e2 = 1j * s * g + c * e
        dg2 = c * dg + 1j * s * de + dphi * (1j * e2)
        de2 = 1j * s * dg + c * de + dphi * (1j * g2)
        psi = m.from_angle(np.stack([g2, e2], axis=1))
        dpsi = m.from_angle(np.stack([dg2, de2], axis=1))
        psi, dpsi = m.potential_half(psi), m.potential_half(dpsi)
        psi, dpsi = m.kinetic_half(psi), m.kinetic_half(dpsi)
        w = (1.0 - m.mask ** 2)[None, None, None, :]
        self.base.absorbed = self.base.absorbed + np.sum(w * np.abs(psi) ** 2, axis=(1, 2, 3)) * m.dr
        self.dab = self.dab + np.sum(w * 2.0 * (np.conj(psi) * dpsi).real, axis=(1, 2, 3)) * m.dr
        self.base.psi = psi * m.mask
        self.dpsi = dpsi * m.mask

    def step(self, n, src_value, dsrc_value):
        b = self.base
        cfg = b.cfg
        b.yee.update_H()
        self.dyee.update_H()
        E = b.yee.E[0].reshape(-1)[b.cells] / E_AU
        dE = self.dyee.E[0].reshape(-1)[b.cells] / E_AU
        self._mol_step(E, dE)
        b.d = b.mol.dipole(b.psi)
        dd = _dipole_differential(b.mol, b.psi, self.dpsi)
        P_new = cfg.mol_weight * b.cell_sums(b.d) * EA0 / cfg.dx ** 3
        dP_new = cfg.mol_weight * b.cell_sums(dd) * EA0 / cfg.dx ** 3
        J = (P_new - b.P) / cfg.dt
        dJ = (dP_new - self.dP) / cfg.dt
        b.P, self.dP = P_new, dP_new
        b.yee.update_E(src_value, cfg.src_k, b.occ, J)
        self.dyee.update_E(dsrc_value, cfg.src_k, b.occ, dJ)

    def objective(self):
        m = self.base.mol
        return float(np.mean(m.dissociated(self.base.psi, self.base.absorbed)))

    def objective_tangent(self):
        m = self.base.mol
        far = m.r > m.r_diss
        t = 2.0 * np.sum((np.conj(self.base.psi[..., far]) * self.dpsi[..., far]).real,
                         axis=(1, 2, 3)) * m.dr + self.dab
        return float(np.mean(t))

    def run(self, src, dsrc):
        for n in range(len(src)):
            self.step(n, src[n], dsrc[n])
        return self.objective(), self.objective_tangent()


def _dipole_differential(m, psi, dpsi):
    """Differential of d = 2 dr sum_r mu12 sum_J c_J Re[conj(g_J) e_{J+1} +
    conj(g_{J+1}) e_J] along dpsi."""
    g, e, dg, de = psi[:, 0], psi[:, 1], dpsi[:, 0], dpsi[:, 1]

    def form(ag, ae, bg, be):
        t = (np.conj(ag[:, :-1]) * be[:, 1:] + np.conj(ag[:, 1:]) * be[:, :-1]).real
        t = np.sum(m.cj[None, :, None] * t, axis=1)
        return 2.0 * m.dr * np.sum(m.mu12[None, :] * t, axis=1)

    return form(dg, de, g, e) + form(g, e, dg, de)


def source_derivatives(cfg, n_steps, knots=None, omega=None):
    """d src[n] / d p for p = (knot_0 .. knot_63, omega): array [n_params, n_steps]
    in V/m per parameter unit, for E_inc(t) = A(t) cos(omega t)."""
    from workloads.pulses import envelope_basis, knot_values, source_times
    from workloads import units as U
    t = source_times(cfg, 0, n_steps)
    a = knot_values(cfg) if knots is None else np.asarray(knots)
    w = cfg.omega if omega is None else omega
    h = envelope_basis(cfg, t)                       # [n_steps, n_knots]
    A = h @ a
    out = np.zeros((cfg.n_knots + 1, n_steps))
    out[:cfg.n_knots] = (h * np.cos(w * t)[:, None]).T * U.E_AU
    out[cfg.n_knots] = -A * t * np.sin(w * t) * U.E_AU
    return out
