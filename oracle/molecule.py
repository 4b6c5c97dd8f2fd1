"""Oracle: two-state ro-vibrational wavepacket step for a batch of molecules.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (section "Efficient numerical implementation of quantum dynamics of
ensembles of molecules ...", Eqs. (3)-(5)): each nuclear wavefunction on the
ground (g) and excited (e) surface is expanded in normalised rotational
functions D^J_{0,0} (m = 0 only), giving radial channels xi_{s,J}(r).  Eq. (5)
gives each channel the Hamiltonian -(1/2mu)(d^2/dr^2 - J(J+1)/r^2) + U_s(r);
Eq. (4) couples g and e through -d_ge(r) E cos(theta) with the field along
the quantisation axis.  The paper propagates Eq. (4) with a split-operator
method using FFTs and integrates the angular part analytically.

Realisation written here, all in complex128, in the order of a symmetric
(Strang) splitting:
    psi <- K_half psi     kinetic half step, FFT along r
    psi <- V_half psi     potential + centrifugal half phase
    psi <- C(E) psi       dipole coupling, exact on the truncated J basis via
                          the Gauss-Legendre angular grid (angular DVR)
    psi <- V_half psi
    psi <- K_half psi
    absorbed += removed norm; psi <- m(r) psi      (edge absorber)

Array layout: psi[mol, s, J, r] complex128 with s in {0: g, 1: e}.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft
from numpy.polynomial.legendre import leggauss
from scipy.special import eval_legendre


def coupling_cj(j_max: int) -> np.ndarray:
    """Matrix elements <J|cos(theta)|J+1> = (J+1)/sqrt((2J+1)(2J+3)) between
    normalised m = 0 rotational functions, J = 0 .. j_max-1 (the selection
    rule Delta J = +-1 of the paper's model)."""
    J = np.arange(j_max, dtype=np.float64)
    return (J + 1.0) / np.sqrt((2.0 * J + 1.0) * (2.0 * J + 3.0))


class MoleculeModel:
    """Grid, operators and one split-operator step of Eqs. (4)-(5)."""

    def __init__(self, n_r, r_min, r_max, j_max, mass, dt, U_g, U_e, mu12,
                 absorb_width=2.0, r_diss=8.0):
        self.n_r = int(n_r)
        self.n_j = int(j_max) + 1
        self.j_max = int(j_max)
        self.mass = float(mass)
        self.dt = float(dt)
        self.r_min = float(r_min)
        self.r_max = float(r_max)
        self.dr = (self.r_max - self.r_min) / self.n_r
        self.r = self.r_min + self.dr * np.arange(self.n_r, dtype=np.float64)
        self.r_diss = float(r_diss)
        self.U = np.stack([np.asarray(U_g, np.float64), np.asarray(U_e, np.float64)])
        self.mu12 = np.asarray(mu12, dtype=np.float64)

        # momenta of the periodic radial grid; forward DFT exp(-2 pi i m k / N)
        m = np.arange(self.n_r)
        m_signed = np.where(m < self.n_r // 2, m, m - self.n_r)
        self.kappa = 2.0 * np.pi * m_signed / (self.n_r * self.dr)
        # kinetic half step: exp(-i (kappa^2 / 2 mu) dt / 2)
        self.kin_half = np.exp(-1j * self.kappa ** 2 * self.dt / (4.0 * self.mass))

        # potential + centrifugal half phase, Eq. (5): exp(-i V_{s,J}(r) dt / 2)
        J = np.arange(self.n_j, dtype=np.float64)
        cent = J[:, None] * (J[:, None] + 1.0) / (2.0 * self.mass * self.r[None, :] ** 2)
        V = self.U[:, None, :] + cent[None, :, :]
        self.v_half = np.exp(-1j * V * self.dt / 2.0)          # [2, nJ, nr]

        # angular grid: Gauss-Legendre nodes x_k = cos(theta_k), weights w_k,
        # T[k, J] = sqrt(w_k) sqrt((2J+1)/2) P_J(x_k)
        x, w = leggauss(self.n_j)
        self.x = x
        self.w = w
        P = np.stack([eval_legendre(j, x) for j in range(self.n_j)], axis=1)   # [k, J]
        self.T = np.sqrt(w)[:, None] * np.sqrt((2.0 * J + 1.0) / 2.0)[None, :] * P

        # edge absorber: 1 below r_a = r_max - width, cos(...)^(1/8) above
        self.mask = np.ones(self.n_r)
        if absorb_width > 0.0:
            ra = self.r_max - absorb_width
            sel = self.r >= ra
            self.mask[sel] = np.cos(np.pi * (self.r[sel] - ra) / (2.0 * absorb_width)) ** 0.125

        self.cj = coupling_cj(self.j_max)

    # ------------------------------------------------------------------ factors
    def kinetic_half(self, psi):
        """F^-1 diag(exp(-i kappa^2 dt / 4 mu)) F along r, per (mol, s, J) line
        (forward transform exp(-2 pi i m k / N), inverse with 1/N; the batch
        of lines spread over all host threads)."""
        return sfft.ifft(self.kin_half * sfft.fft(psi, axis=-1, workers=-1), axis=-1, workers=-1)

    def potential_half(self, psi):
        return psi * self.v_half[None]

    def to_angle(self, psi):
        """Phi[mol, s, k, r] = sum_J T[k, J] psi[mol, s, J, r]."""
        return np.einsum("kj,msjr->mskr", self.T, psi, optimize=True)

    def from_angle(self, phi):
        """psi[mol, s, J, r] = sum_k T[k, J] Phi[mol, s, k, r] (T is orthogonal)."""
        return np.einsum("kj,mskr->msjr", self.T, phi, optimize=True)

    def rotation_angle(self, E):
        """phi[mol, k, r] = mu12(r) x_k E_mol dt: the angle of the exact 2x2
        propagator exp(i phi sigma_x) of H_int = -mu12(r) cos(theta) E sigma_x
        at each angular node, Eq. (4) with the field along the quantisation
        axis."""
        E = np.asarray(E, dtype=np.float64)
        return (self.mu12[None, None, :] * self.x[None, :, None]
                * E[:, None, None] * self.dt)

    def coupling(self, psi, E):
        """exp(-i H_int dt) on the truncated J basis: J -> angle, rotate each
        (k, r) point, angle -> J."""
        phi_ang = self.rotation_angle(E)
        c = np.cos(phi_ang)
        s = np.sin(phi_ang)
        Phi = self.to_angle(psi)
        g = Phi[:, 0]
        e = Phi[:, 1]
        g2 = c * g + 1j * s * e
        e2 = 1j * s * g + c * e
        return self.from_angle(np.stack([g2, e2], axis=1))

    def absorb(self, psi, absorbed):
        """Accumulate sum (1 - m^2)|psi|^2 dr per molecule, then psi *= m."""
        lost = np.sum((1.0 - self.mask ** 2)[None, None, None, :] * np.abs(psi) ** 2,
                      axis=(1, 2, 3)) * self.dr
        return psi * self.mask[None, None, None, :], absorbed + lost

    def step(self, psi, E, absorbed):
        """One molecular time step under the field E (per molecule, au),
        held constant over the step.  Returns (psi, absorbed)."""
        psi = self.kinetic_half(psi)
        psi = self.potential_half(psi)
        psi = self.coupling(psi, E)
        psi = self.potential_half(psi)
        psi = self.kinetic_half(psi)
        return self.absorb(psi, absorbed)

    # ----------------------------------------------------------------- readouts
    def dipole(self, psi):
        """d = <psi| mu12(r) cos(theta) sigma_x |psi> (e a0) per molecule:
        2 dr sum_r mu12 sum_J c_J Re[conj(g_J) e_{J+1} + conj(g_{J+1}) e_J]."""
        g = psi[:, 0]
        e = psi[:, 1]
        t = (np.conj(g[:, :-1]) * e[:, 1:] + np.conj(g[:, 1:]) * e[:, :-1]).real
        t = np.sum(self.cj[None, :, None] * t, axis=1)          # [mol, r]
        return 2.0 * self.dr * np.sum(self.mu12[None, :] * t, axis=1)

    def norm(self, psi):
        return np.sum(np.abs(psi) ** 2, axis=(1, 2, 3)) * self.dr

    def dissociated(self, psi, absorbed):
        """Norm beyond r_diss (both states, strict r > r_diss) plus the norm
        already removed by the absorber."""
        far = self.r > self.r_diss
        return np.sum(np.abs(psi[..., far]) ** 2, axis=(1, 2, 3)) * self.dr + absorbed

    def excited_mean_r(self, psi):
        """<R>_e = <chi_e|R|chi_e> / <chi_e|chi_e>, Eq. (8), per molecule."""
        pe = np.sum(np.abs(psi[:, 1]) ** 2, axis=1)
        return np.sum(pe * self.r[None, :], axis=1) / np.sum(pe, axis=1)

    def excited_r_moments(self, psi):
        """Per molecule <chi_e|R|chi_e> and <chi_e|chi_e> (both states' J
        lines summed over the excited state, times dr); the ensemble value
        of Eq. (8) is sum(first) / sum(second), the excited population
        weighting each molecule."""
        pe = np.sum(np.abs(psi[:, 1]) ** 2, axis=1)
        return (np.sum(pe * self.r[None, :], axis=1) * self.dr, np.sum(pe, axis=1) * self.dr)

    # ------------------------------------------------------------------- state
    def initial_state(self, n_mol, radial):
        """All molecules in (g, J=0) with the given radial function."""
        psi = np.zeros((n_mol, 2, self.n_j, self.n_r), dtype=np.complex128)
        psi[:, 0, 0, :] = np.asarray(radial)
        return psi


def model_from_config(cfg, U_g, U_e, mu12, dt_au=None):
    """The molecular model of a workload; dt_au overrides the step (the
    multi-rate scheme steps molecules by a multiple of the field step)."""
    return MoleculeModel(cfg.n_r, cfg.r_min, cfg.r_max, cfg.j_max, cfg.mass,
                         cfg.dt_au if dt_au is None else dt_au,
                         U_g, U_e, mu12, cfg.absorb_width, cfg.r_diss)
