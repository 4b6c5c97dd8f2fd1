"""Pins of the oracle's molecular step against what the physics fixes.

Each test compares the oracle with something other than itself: closed forms
(plane waves, the free Gaussian, Morse levels, Rabi oscillation), exact
identities of Gauss-Legendre quadrature, angular-momentum matrix elements
obtained by numerical quadrature, and brute-force matrix exponentials.
"""

import math

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import eval_legendre

from oracle.molecule import MoleculeModel


def _model(n_r=64, j_max=2, mass=1.0e4, dt=0.3, absorb=0.0, U=None, mu=None,
           r_min=1.0, r_max=12.0):
    r = r_min + (r_max - r_min) / n_r * np.arange(n_r)
    if U is None:
        U = (0.17 * (1 - np.exp(-(r - 2.0))) ** 2, 0.17 + 0.3 * np.exp(-1.2 * (r - 2.0)))
    if mu is None:
        mu = np.exp(-0.1 * (r - 2.0) ** 2)
    return MoleculeModel(n_r, r_min, r_max, j_max, mass, dt, U[0], U[1], mu,
                         absorb_width=absorb)


def _rand_state(rng, m, n_mol):
    psi = rng.standard_normal((n_mol, 2, m.n_j, m.n_r)) + 1j * rng.standard_normal(
        (n_mol, 2, m.n_j, m.n_r))
    nrm = np.sqrt(np.sum(np.abs(psi) ** 2, axis=(1, 2, 3)) * m.dr)
    return psi / nrm[:, None, None, None]


# ---------------------------------------------------------------- kinetic part
def test_kinetic_half_on_plane_waves():
    """exp(i kappa_m r) is an eigenfunction of -(1/2mu) d^2/dr^2 on the periodic
    grid with eigenvalue kappa_m^2/2mu, kappa_m = 2 pi m / L; K_half multiplies
    it by exp(-i kappa_m^2 dt / (4 mu))."""
    m = _model(n_r=32, dt=7.0, mass=3.0)
    L = m.n_r * m.dr
    for mm in [0, 1, 5, -3, 15, -16]:
        kap = 2 * math.pi * mm / L
        wave = np.exp(1j * kap * (m.r - m.r_min))
        psi = np.zeros((1, 2, m.n_j, m.n_r), complex)
        psi[0, 1, 2] = wave
        out = m.kinetic_half(psi)
        expect = wave * np.exp(-1j * kap ** 2 * m.dt / (4 * m.mass))
        np.testing.assert_allclose(out[0, 1, 2], expect, atol=1e-13)
        assert np.abs(out[0, 0]).max() < 1e-15


def test_kinetic_free_gaussian_closed_form():
    """A free Gaussian spreads as the textbook closed form
    psi(r,t) = (2 pi s^2)^(-1/4) (1 + i tau)^(-1/2) exp(-(r-r0)^2 / (4 s^2 (1 + i tau))),
    tau = t / (2 mu s^2); one K_half advances t by dt/2."""
    mass, s, r0 = 2.0e3, 0.4, 6.5
    dt = 2 * (2 * mass * s * s) * 0.7          # K_half gives tau = 0.7
    m = _model(n_r=256, dt=dt, mass=mass)

    def gauss(t):
        tau = t / (2 * mass * s * s)
        return (2 * math.pi * s * s) ** -0.25 / np.sqrt(1 + 1j * tau) * np.exp(
            -(m.r - r0) ** 2 / (4 * s * s * (1 + 1j * tau)))

    psi = np.zeros((1, 2, m.n_j, m.n_r), complex)
    psi[0, 0, 0] = gauss(0.0)
    out = m.kinetic_half(psi)
    np.testing.assert_allclose(out[0, 0, 0], gauss(dt / 2), atol=1e-10)
    # the opposite time direction gives a clearly different packet
    assert np.abs(out[0, 0, 0] - gauss(-dt / 2)).max() > 1e-3


# ----------------------------------------------------------- Morse eigenvalues
def _step_matrix(m, E=0.0, s=0, J=0):
    """Columns = oracle step applied to unit vectors in one (s, J) channel."""
    n = m.n_r
    psi = np.zeros((n, 2, m.n_j, n), complex)
    for i in range(n):
        psi[i, s, J, i] = 1.0
    out, _ = m.step(psi, np.full(n, E), np.zeros(n))
    return out[:, s, J, :].T


def _morse_levels(D, a, mass, nv):
    w0 = a * math.sqrt(2 * D / mass)
    return np.array([w0 * (v + 0.5) - (w0 * (v + 0.5)) ** 2 / (4 * D) for v in range(nv)])


@pytest.mark.parametrize("n_r", [128, 256])
def test_morse_levels_from_step_eigenphases(n_r):
    """Field free, J = 0: the step is exp(-i H_eff dt) with H_eff = H + O(dt^2);
    its lowest eigenphases reproduce the closed-form Morse levels
    E_v = w0 (v+1/2) - (w0 (v+1/2))^2 / 4D, w0 = a sqrt(2D/mu); the residual
    shrinks ~4x when dt halves (second-order splitting)."""
    D, a, re, mass = 0.17, 1.0, 2.0, 1.0e4
    exact = _morse_levels(D, a, mass, 4)
    errs = []
    for dt in (0.34475, 0.34475 / 2):
        r = 1.0 + 11.0 / n_r * np.arange(n_r)
        ug = D * (1 - np.exp(-a * (r - re))) ** 2
        m = MoleculeModel(n_r, 1.0, 12.0, 0, mass, dt, ug, ug + 1.0, np.zeros(n_r),
                          absorb_width=0.0)
        Umat = _step_matrix(m)
        ev = np.linalg.eigvals(Umat)
        np.testing.assert_allclose(np.abs(ev), 1.0, atol=1e-12)
        eps = np.sort(-np.angle(ev) / dt)
        errs.append(np.abs(eps[:4] - exact) / exact)
    assert errs[0].max() < 5e-6, errs[0]
    ratio = errs[0][:2] / errs[1][:2]
    assert np.all((ratio > 3.0) & (ratio < 5.0)), ratio


# ------------------------------------------------------------------ unitarity
def test_norm_conserved_without_absorber():
    rng = np.random.default_rng(1)
    m = _model(n_r=128, j_max=4, dt=0.34475, absorb=0.0)
    psi = _rand_state(rng, m, 6)
    E = rng.standard_normal(6) * 0.05
    ab = np.zeros(6)
    for _ in range(40):
        psi, ab = m.step(psi, E, ab)
    np.testing.assert_allclose(m.norm(psi), 1.0, atol=1e-13)
    assert np.all(ab == 0.0)


def test_norm_plus_absorbed_is_one():
    """An outgoing packet is removed by the absorber; what leaves the grid is
    exactly what the accumulator records."""
    m = _model(n_r=256, j_max=2, mass=1.0e3, dt=0.5, absorb=2.0)
    k0 = 8.0
    psi = np.zeros((2, 2, m.n_j, m.n_r), complex)
    packet = np.exp(-(m.r - 8.5) ** 2 / 0.5 + 1j * k0 * m.r)
    psi[0, 0, 1] = packet
    psi[1, 1, 2] = packet
    psi /= np.sqrt(m.norm(psi))[:, None, None, None]
    ab = np.zeros(2)
    for _ in range(600):
        psi, ab = m.step(psi, np.array([0.01, -0.02]), ab)
    assert ab.min() > 0.5                       # most of it has been absorbed
    np.testing.assert_allclose(m.norm(psi) + ab, 1.0, atol=1e-13)


# --------------------------------------------------------------- angular DVR
def _cos_matrix_by_quadrature(n_j):
    """<J|cos(theta)|J'> of normalised m=0 functions sqrt((2J+1)/2) P_J(x),
    by a 40-point Gauss-Legendre integration over x = cos(theta) (exact for
    the polynomial degrees involved)."""
    x, w = np.polynomial.legendre.leggauss(40)
    f = np.stack([np.sqrt((2 * j + 1) / 2.0) * eval_legendre(j, x) for j in range(n_j)])
    return (f * x * w) @ f.T


@pytest.mark.parametrize("j_max", [1, 4, 6, 10])
def test_dvr_is_exact_on_truncated_basis(j_max):
    m = _model(n_r=16, j_max=j_max)
    n = m.n_j
    np.testing.assert_allclose(m.T.T @ m.T, np.eye(n), atol=1e-14)
    C = _cos_matrix_by_quadrature(n)
    np.testing.assert_allclose(m.T.T @ np.diag(m.x) @ m.T, C, atol=1e-13)
    # and the closed form of the off-diagonal elements
    J = np.arange(j_max)
    np.testing.assert_allclose(np.diag(C, 1), (J + 1) / np.sqrt((2 * J + 1) * (2 * J + 3)),
                               atol=1e-14)


def _dense_coupling(m, r_index, E):
    """exp(+i mu12 E dt C (x) sigma_x) on the (s, J) space at one radial point,
    with C from quadrature."""
    C = _cos_matrix_by_quadrature(m.n_j)
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    H = -m.mu12[r_index] * E * np.kron(sx, C)           # index s*nJ + J
    return expm(-1j * H * m.dt)


def test_coupling_matches_dense_expm():
    rng = np.random.default_rng(2)
    m = _model(n_r=16, j_max=5, dt=0.7)
    psi = _rand_state(rng, m, 3)
    E = np.array([0.3, -1.1, 0.05])
    out = m.coupling(psi, E)
    for i in range(3):
        for r in range(m.n_r):
            U = _dense_coupling(m, r, E[i])
            v = psi[i, :, :, r].reshape(-1)
            np.testing.assert_allclose(out[i, :, :, r].reshape(-1), U @ v, atol=1e-13)


# ------------------------------------------------------ whole step vs expm
def _dense_parts(m, E):
    """(H_kin, H_pot, H_int) as dense matrices on index (s, J, r) ->
    (s*nJ + J)*nr + r: -(1/2mu) d2/dr2 built from the DFT matrix, the diagonal
    U_s(r) + J(J+1)/(2 mu r^2), and -mu12(r) E cos(theta) sigma_x with
    cos(theta) from quadrature."""
    n = m.n_r
    L = n * m.dr
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    k = 2 * np.pi * np.fft.fftfreq(n, d=1.0) * n / L
    Kr = (np.conj(F).T @ np.diag(k ** 2) @ F / n) / (2 * m.mass)
    nj = m.n_j
    dim = 2 * nj * n
    Hk = np.zeros((dim, dim), complex)
    Hv = np.zeros((dim, dim), complex)
    Hc = np.zeros((dim, dim), complex)
    C = _cos_matrix_by_quadrature(nj)
    for s in range(2):
        for J in range(nj):
            o = (s * nj + J) * n
            Hk[o:o + n, o:o + n] = Kr
            Hv[o:o + n, o:o + n] = np.diag(m.U[s] + J * (J + 1) / (2 * m.mass * m.r ** 2))
    for J in range(nj):
        for J2 in range(nj):
            blk = -E * np.diag(m.mu12) * C[J, J2]
            og = J * n
            oe = (nj + J2) * n
            Hc[og:og + n, oe:oe + n] += blk
            Hc[oe:oe + n, og:og + n] += blk
    return Hk, Hv, Hc


def test_step_equals_product_of_exact_factors_and_is_second_order():
    rng = np.random.default_rng(3)
    n_r, j_max, mass = 16, 2, 1.0
    r = 1.0 + 11.0 / n_r * np.arange(n_r)
    U = (0.05 * np.sin(r), 0.2 + 0.03 * np.cos(2 * r))
    mu = 0.8 + 0.1 * np.sin(r)
    E = 0.7
    errs = []
    dts = [0.04, 0.02, 0.01]
    psi0 = None
    for dt in dts:
        m = MoleculeModel(n_r, 1.0, 12.0, j_max, mass, dt, U[0], U[1], mu, absorb_width=0.0)
        if psi0 is None:
            psi0 = _rand_state(rng, m, 1)
        psi = psi0.copy()
        v = psi[0].reshape(-1)
        out, _ = m.step(psi, np.array([E]), np.zeros(1))
        Hk, Hv, Hc = _dense_parts(m, E)
        Kh = expm(-1j * Hk * dt / 2)
        Vh = expm(-1j * Hv * dt / 2)
        Cf = expm(-1j * Hc * dt)
        strang = Kh @ Vh @ Cf @ Vh @ Kh
        np.testing.assert_allclose(out[0].reshape(-1), strang @ v, atol=1e-12)
        exact = expm(-1j * (Hk + Hv + Hc) * dt) @ v
        errs.append(np.linalg.norm(out[0].reshape(-1) - exact) * math.sqrt(m.dr))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(dts))
    assert np.all((slopes > 2.7) & (slopes < 3.3)), slopes


# ------------------------------------------------------------- Rabi limit
def test_two_level_rabi_weak_field():
    """J_max = 1, flat surfaces 0 and Delta, constant dipole, huge mass (no
    nuclear motion): (g,0) <-> (e,1) is a two-level system with coupling
    mu E cos(Delta t) / sqrt(3); in the weak-field limit the excited
    population follows sin^2(Omega t / 2), Omega = mu E0 / sqrt(3)."""
    n_r = 8
    Delta = 0.1
    Omega = 4e-3 * Delta
    mu0 = 1.0
    E0 = Omega * math.sqrt(3) / mu0
    dt = 0.5
    m = MoleculeModel(n_r, 1.0, 12.0, 1, 1.0e12, dt, np.zeros(n_r), np.full(n_r, Delta),
                      np.full(n_r, mu0), absorb_width=0.0)
    psi = np.zeros((1, 2, 2, n_r), complex)
    psi[0, 0, 0, :] = 1.0 / math.sqrt(n_r * m.dr)
    ab = np.zeros(1)
    n_steps = int(round(math.pi / Omega / dt))
    checks = {n_steps // 4, n_steps // 2, n_steps}
    for n in range(1, n_steps + 1):
        t_mid = (n - 0.5) * dt
        psi, ab = m.step(psi, np.array([E0 * math.cos(Delta * t_mid)]), ab)
        if n in checks:
            pe = np.sum(np.abs(psi[0, 1]) ** 2) * m.dr
            expect = math.sin(Omega * n * dt / 2) ** 2
            assert abs(pe - expect) < 1e-2, (n, pe, expect)
            # the other pair (g,1)/(e,0) stays empty
            assert np.sum(np.abs(psi[0, 0, 1]) ** 2 + np.abs(psi[0, 1, 0]) ** 2) < 1e-20


# ------------------------------------------------------------ dipole readout
def test_dipole_readout_matches_dense_operator():
    """d = dr psi^H (mu12 cos(theta) sigma_x) psi with cos(theta) from quadrature."""
    rng = np.random.default_rng(4)
    m = _model(n_r=16, j_max=4)
    psi = _rand_state(rng, m, 2)
    d = m.dipole(psi)
    C = _cos_matrix_by_quadrature(m.n_j)
    for i in range(2):
        g = psi[i, 0]
        e = psi[i, 1]
        val = 0.0
        for r in range(m.n_r):
            val += m.mu12[r] * (np.conj(g[:, r]) @ C @ e[:, r] + np.conj(e[:, r]) @ C @ g[:, r]).real
        np.testing.assert_allclose(d[i], val * m.dr, rtol=1e-13)


def test_constant_dipole_is_special_case():
    """A flat dipole table (the paper's constant 10 D) goes through the same
    path: the coupling then commutes with r and equals the per-r expm."""
    rng = np.random.default_rng(5)
    mu_const = 10.0 * 0.3934302                    # 10 debye in e a0
    m = _model(n_r=16, j_max=3, mu=np.full(16, mu_const), dt=0.1)
    psi = _rand_state(rng, m, 1)
    out = m.coupling(psi, np.array([1e-3]))
    U = _dense_coupling(m, 0, 1e-3)
    for r in range(m.n_r):
        np.testing.assert_allclose(out[0, :, :, r].reshape(-1), U @ psi[0, :, :, r].reshape(-1),
                                   atol=1e-14)


def test_dissociation_yield_identity():
    """With the absorber beyond r_diss, yield = 1 - norm(r <= r_diss) exactly
    for a normalised start."""
    m = _model(n_r=256, j_max=2, mass=1.0e3, dt=0.5, absorb=2.0)
    psi = np.zeros((1, 2, m.n_j, m.n_r), complex)
    psi[0, 1, 1] = np.exp(-(m.r - 6.0) ** 2 + 25j * m.r)
    psi /= math.sqrt(m.norm(psi)[0])
    ab = np.zeros(1)
    for _ in range(300):
        psi, ab = m.step(psi, np.array([0.0]), ab)
    near = np.sum(np.abs(psi[..., m.r <= m.r_diss]) ** 2) * m.dr
    np.testing.assert_allclose(m.dissociated(psi, ab)[0], 1.0 - near, atol=1e-13)
    assert m.dissociated(psi, ab)[0] > 0.1


def test_excited_mean_r_of_symmetric_packets():
    """Eq. (8): a packet whose |chi_e|^2 is symmetric about a grid point r0
    has <R>_e = r0 exactly; the ensemble value weights molecules by their
    excited population; the ground state does not enter."""
    m = _model(n_r=128, j_max=2)
    psi = np.zeros((2, 2, m.n_j, m.n_r), complex)
    k0, k1 = 40, 70
    for mol, k in ((0, k0), (1, k1)):
        g = np.exp(-((np.arange(m.n_r) - k) / 4.0) ** 2)
        psi[mol, 1, 1] = g * (0.3 if mol == 0 else 0.9)
        psi[mol, 1, 2] = 0.5j * g
        psi[mol, 0, 0] = np.roll(g, 10)          # ground population elsewhere
    mean = m.excited_mean_r(psi)
    np.testing.assert_allclose(mean, [m.r[k0], m.r[k1]], rtol=1e-13)
    num, pop = m.excited_r_moments(psi)
    np.testing.assert_allclose(num / pop, mean, rtol=1e-13)
    w = pop / pop.sum()
    np.testing.assert_allclose(num.sum() / pop.sum(), w[0] * m.r[k0] + w[1] * m.r[k1], rtol=1e-13)
    np.testing.assert_allclose(pop, np.sum(np.abs(psi[:, 1]) ** 2, axis=(1, 2)) * m.dr, rtol=1e-13)
