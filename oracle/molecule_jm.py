"""Oracle: the molecular step in the full rotational basis |j, m> with all
three field components.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (3) expands each electronic state's wavefunction over the rotational
functions Y_jm of the molecular axis; with a field of any direction the
interaction -mu12(r) (E . d) sigma_x, d the unit vector along the molecular
axis, couples j to j +- 1 and m to m and m +- 1 (the X, Y, Z direction-cosine
elements of the paper's angular integration).  Here the basis is truncated at
j <= j_max with all m = -j..j, ordered b = j^2 + (m + j).

The split-operator step is the one of oracle.molecule (K/2 V/2 C V/2 K/2,
then the absorber) with
  - V/2 depending on (s, j): U_s(r) + j(j+1)/(2 mu r^2);
  - C = exp(i mu12(r) dt sigma_x (x) A(E)), A = sum_c E_c D_c, the exact
    exponential on the truncated basis (the reading used for m = 0 as well),
    evaluated from the eigen-decomposition of the Hermitian A (a library
    routine);
  - the direction-cosine matrices D_c[b', b] = <Y_b'| d_c |Y_b> by product
    quadrature of the spherical harmonics (Gauss-Legendre in cos(theta) times
    a uniform azimuthal grid, exact for these polynomial integrands).
The dipole is the vector d_c = <psi| mu12 sigma_x (x) D_c |psi>.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft
from numpy.polynomial.legendre import leggauss
from scipy.special import sph_harm_y


def jm_basis(j_max):
    return [(j, m) for j in range(j_max + 1) for m in range(-j, j + 1)]


def direction_cosines(j_max):
    """D[c, b', b] = int conj(Y_b') d_c Y_b dOmega, c = x, y, z."""
    basis = jm_basis(j_max)
    n_t = 2 * j_max + 4
    n_p = 2 * j_max + 4
    x, w = leggauss(n_t)
    theta = np.arccos(x)
    phi = 2.0 * np.pi * np.arange(n_p) / n_p
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    W = w[:, None] * (2.0 * np.pi / n_p) * np.ones_like(PH)
    Y = np.stack([sph_harm_y(j, m, TH, PH) for (j, m) in basis])     # [b, t, p]
    d = [np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)]
    D = np.zeros((3, len(basis), len(basis)), complex)
    for c in range(3):
        D[c] = np.einsum("atp,tp,btp->ab", np.conj(Y), W * d[c], Y)
    return D


class MoleculeJM:
    def __init__(self, n_r, r_min, r_max, j_max, mass, dt, U_g, U_e, mu12,
                 absorb_width=2.0, r_diss=8.0):
        self.n_r = int(n_r)
        self.j_max = int(j_max)
        self.basis = jm_basis(self.j_max)
        self.n_b = len(self.basis)
        self.mass = float(mass)
        self.dt = float(dt)
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.dr = (self.r_max - self.r_min) / self.n_r
        self.r = self.r_min + self.dr * np.arange(self.n_r, dtype=np.float64)
        self.r_diss = float(r_diss)
        self.U = np.stack([np.asarray(U_g, np.float64), np.asarray(U_e, np.float64)])
        self.mu12 = np.asarray(mu12, dtype=np.float64)
        m = np.arange(self.n_r)
        m_signed = np.where(m < self.n_r // 2, m, m - self.n_r)
        self.kappa = 2.0 * np.pi * m_signed / (self.n_r * self.dr)
        self.kin_half = np.exp(-1j * self.kappa ** 2 * self.dt / (4.0 * self.mass))
        jb = np.array([j for (j, _) in self.basis], dtype=np.float64)
        cent = jb[:, None] * (jb[:, None] + 1.0) / (2.0 * self.mass * self.r[None, :] ** 2)
        self.v_half = np.exp(-1j * (self.U[:, None, :] + cent[None]) * self.dt / 2.0)   # [2, nb, nr]
        self.D = direction_cosines(self.j_max)
        self.mask = np.ones(self.n_r)
        if absorb_width > 0.0:
            ra = self.r_max - absorb_width
            sel = self.r >= ra
            self.mask[sel] = np.cos(np.pi * (self.r[sel] - ra) / (2.0 * absorb_width)) ** 0.125

    def kinetic_half(self, psi):
        return sfft.ifft(self.kin_half * sfft.fft(psi, axis=-1, workers=-1), axis=-1, workers=-1)

    def potential_half(self, psi):
        return psi * self.v_half[None]

    def coupling(self, psi, E3):
        """psi[mol, s, b, r] -> exp(i mu12(r) dt sigma_x (x) A) psi per (mol, r),
        A = sum_c E_c D_c, E3[mol, c] in au."""
        out = np.empty_like(psi)
        for i in range(psi.shape[0]):
            A = np.einsum("c,cab->ab", np.asarray(E3[i], np.float64), self.D)
            lam, W = np.linalg.eigh(A)
            ph = self.mu12[:, None] * self.dt * lam[None, :]          # [r, k]
            c, s = np.cos(ph), np.sin(ph)
            g = np.conj(W).T @ psi[i, 0]                               # [k, r]
            e = np.conj(W).T @ psi[i, 1]
            g2 = c.T * g + 1j * s.T * e
            e2 = 1j * s.T * g + c.T * e
            out[i, 0] = W @ g2
            out[i, 1] = W @ e2
        return out

    def absorb(self, psi, absorbed):
        lost = np.sum((1.0 - self.mask ** 2)[None, None, None, :] * np.abs(psi) ** 2,
                      axis=(1, 2, 3)) * self.dr
        return psi * self.mask[None, None, None, :], absorbed + lost

    def step(self, psi, E3, absorbed):
        psi = self.kinetic_half(psi)
        psi = self.potential_half(psi)
        psi = self.coupling(psi, E3)
        psi = self.potential_half(psi)
        psi = self.kinetic_half(psi)
        return self.absorb(psi, absorbed)

    def dipole(self, psi):
        """d[mol, c] = <psi| mu12(r) sigma_x (x) D_c |psi> (e a0) =
        2 dr sum_r mu12 Re <g(r)| D_c |e(r)>."""
        g, e = psi[:, 0], psi[:, 1]
        t = np.einsum("mar,cab,mbr->mcr", np.conj(g), self.D, e).real
        return 2.0 * self.dr * np.sum(self.mu12[None, None, :] * t, axis=2)

    def norm(self, psi):
        return np.sum(np.abs(psi) ** 2, axis=(1, 2, 3)) * self.dr

    def dissociated(self, psi, absorbed):
        far = self.r > self.r_diss
        return np.sum(np.abs(psi[..., far]) ** 2, axis=(1, 2, 3)) * self.dr + absorbed

    def initial_state(self, n_mol, radial):
        """All molecules in (g, j = 0, m = 0) with the given radial function."""
        psi = np.zeros((n_mol, 2, self.n_b, self.n_r), dtype=np.complex128)
        psi[:, 0, 0, :] = np.asarray(radial)
        return psi


def jm_model_from_config(cfg, U_g, U_e, mu12, dt_au=None):
    return MoleculeJM(cfg.n_r, cfg.r_min, cfg.r_max, cfg.j_max, cfg.mass,
                      cfg.dt_au if dt_au is None else dt_au, U_g, U_e, mu12,
                      cfg.absorb_width, cfg.r_diss)
