"""Oracle: Yee leap-frog FDTD with a Drude metal, CPML in z, periodic x/y.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "The domain decomposition methodology for FDTD": Maxwell's curl
equations, Eq. (1), are discretised with central differences on the
staggered Yee cell and marched by leap-frog; metals follow the Drude current
of Eq. (2), dJ/dt + gamma J = eps0 Omega_p^2 E; x and y are periodic and z is
terminated by convolutional PMLs; a plane wave excites the structure and the
energy flux through a detection plane is Fourier transformed.

SI units.  Field placement (cell units): E_x (i+1/2, j, k), E_y (i, j+1/2, k),
E_z (i, j, k+1/2), H_x (i, j+1/2, k+1/2), H_y (i+1/2, j, k+1/2),
H_z (i+1/2, j+1/2, k).  Arrays are [k][j][i].  Beyond the CPML the grid ends
on tangential E = 0 (E_x, E_y at k = 0 and at k = nz are held at zero).

Discretisation (the paper gives only the continuous equations):
  H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n
  J_D^{n+1/2} = alpha J_D^{n-1/2} + beta E^n      (centred form of Eq. (2))
  E^{n+1} = E^n + dt/(eps0 eps_r) [curl H^{n+1/2} - J_D^{n+1/2} - J_mol - J_src]
with alpha = (1 - g dt/2)/(1 + g dt/2), beta = eps0 wp^2 dt/(1 + g dt/2), and
the CPML stretching (1/kappa) d/dz + psi, psi <- b psi + a d/dz.
"""

from __future__ import annotations

import numpy as np

C0 = 299792458.0
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
ETA0 = 376.730313668


def cpml_profile(nz, npml, m, sigma_lo, sigma_hi, kappa_max, alpha_max, dt, offset):
    """(b, a, kappa) along z at positions z = k + offset (cell units).

    The graded layer occupies depth d in (0, npml] measured from each inner
    interface (z = npml at the bottom, z = nz - npml at the top):
    sigma = sigma_max (d/npml)^m, kappa = 1 + (kappa_max-1)(d/npml)^m,
    alpha = alpha_max (1 - d/npml)."""
    z = np.arange(nz, dtype=np.float64) + offset
    b = np.ones(nz)
    a = np.zeros(nz)
    kap = np.ones(nz)
    if npml == 0:
        return b, a, kap
    for k in range(nz):
        if z[k] < npml:
            d = (npml - z[k]) / npml
            smax = sigma_lo
        elif z[k] > nz - npml:
            d = (z[k] - (nz - npml)) / npml
            smax = sigma_hi
        else:
            continue
        sig = smax * d ** m
        kk = 1.0 + (kappa_max - 1.0) * d ** m
        al = alpha_max * (1.0 - d)
        bb = np.exp(-(sig / kk + al) * dt / EPS0)
        b[k] = bb
        kap[k] = kk
        a[k] = sig * (bb - 1.0) / (sig * kk + kk * kk * al) if sig > 0.0 else 0.0
    return b, a, kap


class Yee:
    def __init__(self, nx, ny, nz, dx, dt, mat, eps_table, wp, gamma, npml,
                 cpml_m=3.0, sigma_lo=0.0, sigma_hi=0.0, kappa_max=1.0, alpha_max=0.0,
                 periodic_z=False, metal_id=2):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dx = float(dx)
        self.dt = float(dt)
        self.periodic_z = periodic_z
        shape = (nz, ny, nx)
        self.E = [np.zeros(shape) for _ in range(3)]
        self.H = [np.zeros(shape) for _ in range(3)]
        self.JD = [np.zeros(shape) for _ in range(3)]
        # CPML auxiliaries (kept on the whole grid; zero outside the layers)
        self.psi_Ex = np.zeros(shape)
        self.psi_Ey = np.zeros(shape)
        self.psi_Hx = np.zeros(shape)
        self.psi_Hy = np.zeros(shape)
        mat = np.asarray(mat)
        eps_table = np.asarray(eps_table, dtype=np.float64)
        self.metal = [mat[c] == metal_id for c in range(3)]
        self.ce = [self.dt / (EPS0 * eps_table[mat[c]]) for c in range(3)]
        self.alpha_d = (1.0 - gamma * dt / 2.0) / (1.0 + gamma * dt / 2.0)
        self.beta_d = EPS0 * wp * wp * dt / (1.0 + gamma * dt / 2.0)
        npml_eff = 0 if periodic_z else npml
        self.bE, self.aE, self.kE = cpml_profile(nz, npml_eff, cpml_m, sigma_lo, sigma_hi,
                                                 kappa_max, alpha_max, dt, 0.0)
        self.bH, self.aH, self.kH = cpml_profile(nz, npml_eff, cpml_m, sigma_lo, sigma_hi,
                                                 kappa_max, alpha_max, dt, 0.5)

    # z neighbours with the tangential-E = 0 termination (or periodic)
    def _up(self, f):
        """f at k+1 (zero beyond the top)."""
        if self.periodic_z:
            return np.roll(f, -1, axis=0)
        g = np.zeros_like(f)
        g[:-1] = f[1:]
        return g

    def _down(self, f):
        """f at k-1 (zero below the bottom)."""
        if self.periodic_z:
            return np.roll(f, 1, axis=0)
        g = np.zeros_like(f)
        g[1:] = f[:-1]
        return g

    def update_H(self):
        Ex, Ey, Ez = self.E
        Hx, Hy, Hz = self.H
        dx = self.dx
        b = self.bH[:, None, None]
        a = self.aH[:, None, None]
        k = self.kH[:, None, None]
        c = self.dt / MU0
        # H_x: curl_x = dEz/dy - dEy/dz
        dEz_dy = (np.roll(Ez, -1, axis=1) - Ez) / dx
        dEy_dz = (self._up(Ey) - Ey) / dx
        self.psi_Hx = b * self.psi_Hx + a * dEy_dz
        Hx -= c * (dEz_dy - (dEy_dz / k + self.psi_Hx))
        # H_y: curl_y = dEx/dz - dEz/dx
        dEx_dz = (self._up(Ex) - Ex) / dx
        dEz_dx = (np.roll(Ez, -1, axis=2) - Ez) / dx
        self.psi_Hy = b * self.psi_Hy + a * dEx_dz
        Hy -= c * ((dEx_dz / k + self.psi_Hy) - dEz_dx)
        # H_z: curl_z = dEy/dx - dEx/dy
        dEy_dx = (np.roll(Ey, -1, axis=2) - Ey) / dx
        dEx_dy = (np.roll(Ex, -1, axis=1) - Ex) / dx
        Hz -= c * (dEy_dx - dEx_dy)

    def update_E(self, src_value=0.0, src_k=None, jmol_cells=None, jmol=None):
        """Advance E by one step.  src_value: E_inc(t_{n+1/2}) in V/m of the
        soft current sheet J_x = -2 E_inc/(eta0 dz) on plane src_k; jmol:
        polarisation current density (A/m^2) added at the flat indices
        jmol_cells, to J_x ([n]) or to each of J_x, J_y, J_z ([3, n])."""
        Hx, Hy, Hz = self.H
        dx = self.dx
        b = self.bE[:, None, None]
        a = self.aE[:, None, None]
        k = self.kE[:, None, None]
        # curl H at the E locations
        dHz_dy = (Hz - np.roll(Hz, 1, axis=1)) / dx
        dHy_dz = (Hy - self._down(Hy)) / dx
        self.psi_Ex = b * self.psi_Ex + a * dHy_dz
        curl_x = dHz_dy - (dHy_dz / k + self.psi_Ex)
        dHx_dz = (Hx - self._down(Hx)) / dx
        dHz_dx = (Hz - np.roll(Hz, 1, axis=2)) / dx
        self.psi_Ey = b * self.psi_Ey + a * dHx_dz
        curl_y = (dHx_dz / k + self.psi_Ey) - dHz_dx
        dHy_dx = (Hy - np.roll(Hy, 1, axis=2)) / dx
        dHx_dy = (Hx - np.roll(Hx, 1, axis=1)) / dx
        curl_z = dHy_dx - dHx_dy
        curls = [curl_x, curl_y, curl_z]

        for c in range(3):
            J = np.zeros_like(self.E[c])
            # Drude current, Eq. (2), centred at step n
            jd = np.where(self.metal[c], self.alpha_d * self.JD[c] + self.beta_d * self.E[c], 0.0)
            self.JD[c] = jd
            J += jd
            if c == 0 and src_k is not None and src_value != 0.0:
                J[src_k] += -2.0 * src_value / (ETA0 * dx)
            if jmol is not None:
                jm = np.asarray(jmol)
                # [n] : current on E_x only; [3, n] : on E_x, E_y, E_z at each
                # cell's own edges (the same flat index in each component array)
                if jm.ndim == 2 or c == 0:
                    Jf = J.reshape(-1)
                    np.add.at(Jf, np.asarray(jmol_cells), jm[c] if jm.ndim == 2 else jm)
            newE = self.E[c] + self.ce[c] * (curls[c] - J)
            if c < 2 and not self.periodic_z:
                newE[0] = 0.0          # tangential E = 0 at the bottom end
            self.E[c] = newE

    def energy(self):
        """Field energy density sum (vacuum, all cells) - used by tests."""
        e = sum(np.sum(f * f) for f in self.E) * EPS0 / 2.0
        h = sum(np.sum(f * f) for f in self.H) * MU0 / 2.0
        return (e + h) * self.dx ** 3


class FluxMonitor:
    """Running DFT of E_x, E_y (at t_{n+1}) and H_x, H_y (at t_{n+1/2},
    averaged over the two planes k-1/2 and k+1/2) on the plane k = mon_k, and
    the plane-averaged z-flux S_z = 1/2 Re(E_x H_y* - E_y H_x*)."""

    def __init__(self, ny, nx, mon_k, omegas, dt, every):
        self.k = mon_k
        self.w = np.asarray(omegas, dtype=np.float64)
        self.dt = dt
        self.every = every
        nf = len(self.w)
        self.Ex = np.zeros((nf, ny, nx), complex)
        self.Ey = np.zeros((nf, ny, nx), complex)
        self.Hx = np.zeros((nf, ny, nx), complex)
        self.Hy = np.zeros((nf, ny, nx), complex)

    def sample(self, yee: Yee, n):
        """Called after step n (fields E^{n+1}, H^{n+1/2})."""
        if (n + 1) % self.every != 0:
            return
        k = self.k
        tE = (n + 1) * self.dt
        tH = (n + 0.5) * self.dt
        wE = np.exp(1j * self.w * tE)[:, None, None] * self.every * self.dt
        wH = np.exp(1j * self.w * tH)[:, None, None] * self.every * self.dt
        hx = 0.5 * (yee.H[0][k - 1] + yee.H[0][k])
        hy = 0.5 * (yee.H[1][k - 1] + yee.H[1][k])
        self.Ex += wE * yee.E[0][k][None]
        self.Ey += wE * yee.E[1][k][None]
        self.Hx += wH * hx[None]
        self.Hy += wH * hy[None]

    def flux(self):
        s = 0.5 * (self.Ex * np.conj(self.Hy) - self.Ey * np.conj(self.Hx)).real
        return s.mean(axis=(1, 2))


def spectra(S_trans, S_inc_side, S_ref):
    """Transmission, reflection and absorption from the net z-fluxes of one
    run and of a vacuum reference run with the same source: S_trans on the
    plane beyond the structure, S_inc_side on a plane between the source and
    the structure (net flux = incident - reflected for plane waves), S_ref the
    reference run's flux on that same incident-side plane.  T = S_trans/S_ref,
    R = 1 - S_inc_side/S_ref, A = 1 - T - R (the spectra of the paper's
    short-pulse technique, section on 3D domain decomposition and Fig. 6a)."""
    T = np.asarray(S_trans) / np.asarray(S_ref)
    R = 1.0 - np.asarray(S_inc_side) / np.asarray(S_ref)
    return T, R, 1.0 - T - R


def yee_from_config(cfg, mat, eps_table, periodic_z=False):
    return Yee(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dt, mat, eps_table, cfg.wp, cfg.gamma,
               cfg.npml, cfg.cpml_m, cfg.sigma_max_lo, cfg.sigma_max_hi,
               cfg.cpml_kappa_max, cfg.cpml_alpha_max, periodic_z=periodic_z)
