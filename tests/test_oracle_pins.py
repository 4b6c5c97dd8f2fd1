"""Pins of three parts of the oracle's molecular model that the other oracle
tests do not reach: the centrifugal term of Eq. (5), the edge absorber, and
the closed-form Morse v = 0 start of the workloads (Eq. (6) family).

Each pin compares with something fixed outside the oracle's own formulas:

* centrifugal term J(J+1)/(2 mu r^2): the rotational structure of the
  rotating Morse oscillator in Pekeris' closed form (Phys. Rev. 45, 98
  (1934)), E(v, J) - E(v, 0) = B_v J(J+1) - D_J [J(J+1)]^2 with
  B_e = 1/(2 mu r_e^2), alpha_e = 6 sqrt(w_e x_e B_e^3)/w_e - 6 B_e^2/w_e,
  B_v = B_e - alpha_e (v + 1/2), D_J = 4 B_e^3 / w_e^2 and the Morse
  w_e = a sqrt(2D/mu), w_e x_e = w_e^2/(4D), read off the field-free step's
  eigenphases in the J channels;
* absorber cos^(1/8): mask values at grid points where the cosine has a
  radical closed form (angles k pi/12), and the norm removed from a flat
  density, against the integral of cos^(1/4) over a quarter period written
  with Gamma functions;
* Morse v = 0: the lowest eigenvector and eigenvalue of the dense Fourier-
  grid Hamiltonian (kinetic operator built from the DFT matrix), and the
  closed-form level w_e/2 - w_e^2/(16 D).

The mutation tests plant the slips these pins exist to catch (a factor 2
or r instead of r^2 in the centrifugal term, J^2 for J(J+1), the exponent 8
for 1/8, lambda +- 1/2 in the Morse function) into copies of the oracle's
tables and check that the pins then fail.
"""

import math

import numpy as np
import pytest
from scipy.special import gamma

from oracle.molecule import MoleculeModel
from workloads import get_config
from workloads.molecule_inputs import morse_v0, potentials

D, A, RE, MASS = 0.17, 1.0, 2.0, 1.0e4
J_MAX = 10
DT = 0.1379          # the SRR workloads' molecular step (au)


# ------------------------------------------------------ rotating Morse (J > 0)
def _pekeris_rotational(v, J):
    """E(v, J) - E(v, 0) of the rotating Morse oscillator (Pekeris)."""
    we = A * math.sqrt(2.0 * D / MASS)
    wexe = we * we / (4.0 * D)
    be = 1.0 / (2.0 * MASS * RE * RE)
    alpha = 6.0 * math.sqrt(wexe * be ** 3) / we - 6.0 * be * be / we
    dj = 4.0 * be ** 3 / (we * we)
    x = J * (J + 1.0)
    return (be - alpha * (v + 0.5)) * x - dj * x * x


def _rot_model(n_r=256):
    r = 1.0 + 11.0 / n_r * np.arange(n_r)
    ug = D * (1.0 - np.exp(-A * (r - RE))) ** 2
    return MoleculeModel(n_r, 1.0, 12.0, J_MAX, MASS, DT, ug, ug + 1.0, np.zeros(n_r),
                         absorb_width=0.0)


def _channel_levels(m, J, n_levels=2):
    """Lowest quasi-energies -arg(eig)/dt of the field-free step restricted to
    the (g, J) channel (the step keeps channels apart without a field)."""
    n = m.n_r
    psi = np.zeros((n, 2, m.n_j, n), complex)
    for i in range(n):
        psi[i, 0, J, i] = 1.0
    out, _ = m.step(psi, np.zeros(n), np.zeros(n))
    ev = np.linalg.eigvals(out[:, 0, J, :].T)
    return np.sort(-np.angle(ev) / m.dt)[:n_levels]


def _rotational_errors(m):
    """Relative error of E(v, J) - E(v, 0), v = 0 and 1, J = 1..10, against
    the closed form."""
    lev = np.array([_channel_levels(m, J) for J in range(J_MAX + 1)])
    err = np.zeros((2, J_MAX))
    for v in range(2):
        for J in range(1, J_MAX + 1):
            exact = _pekeris_rotational(v, J)
            err[v, J - 1] = abs((lev[J, v] - lev[0, v]) - exact) / exact
    return err


def _with_centrifugal(m, cent):
    """A copy of the model's potential half-phase with the centrifugal term
    replaced (the planted mutations)."""
    V = m.U[:, None, :] + cent[None, :, :]
    m.v_half = np.exp(-1j * V * m.dt / 2.0)
    return m


def test_centrifugal_term_against_rotating_morse():
    """J = 1..10 of the v = 0 and v = 1 levels: Pekeris' closed form holds to
    2e-5 (v = 0, measured 6.3e-6) and 2e-4 (v = 1, measured 8.2e-5; the
    closed form drops terms of order gamma_e (v+1/2)^2 J(J+1))."""
    err = _rotational_errors(_rot_model())
    assert err[0].max() < 2e-5, err[0]
    assert err[1].max() < 2e-4, err[1]


@pytest.mark.parametrize("slip", ["factor_2", "r_not_r2", "J_squared", "double_mass"])
def test_centrifugal_pin_catches_planted_slips(slip):
    m = _rot_model()
    J = np.arange(m.n_j, dtype=np.float64)[:, None]
    r = m.r[None, :]
    cent = {
        "factor_2": J * (J + 1.0) / (MASS * r * r),
        "r_not_r2": J * (J + 1.0) / (2.0 * MASS * r),
        "J_squared": J * J / (2.0 * MASS * r * r),
        "double_mass": J * (J + 1.0) / (4.0 * MASS * r * r),
    }[slip]
    err = _rotational_errors(_with_centrifugal(m, cent))
    assert err[0].max() > 1e-2, (slip, err[0].max())


# ------------------------------------------------------------------- absorber
def _mask_model(n_r=36, exponent=None):
    """Radial box [1, 13) with dr = 1/3 and a 2 a0 absorber from r_a = 11:
    grid points sit at r_a + k/3, i.e. at angles k pi/12 of the mask's
    cosine."""
    r = 1.0 + 12.0 / n_r * np.arange(n_r)
    m = MoleculeModel(n_r, 1.0, 13.0, 1, MASS, DT, np.zeros(n_r), np.zeros(n_r), np.zeros(n_r),
                      absorb_width=2.0)
    if exponent is not None:          # planted mutation of the exponent
        sel = r >= 11.0
        m.mask = np.ones(n_r)
        m.mask[sel] = np.cos(np.pi * (r[sel] - 11.0) / 4.0) ** exponent
    return m


# cos(k pi / 12), k = 0..5, as radicals
_COS_K_PI_12 = [1.0, (math.sqrt(6.0) + math.sqrt(2.0)) / 4.0, math.sqrt(3.0) / 2.0,
                math.sqrt(2.0) / 2.0, 0.5, (math.sqrt(6.0) - math.sqrt(2.0)) / 4.0]


def _mask_error(m):
    """Largest deviation of the mask from 1 below r_a and from
    cos(k pi/12)^(1/8) on the six absorber points."""
    k_a = 30                         # r = 1 + 30/3 = 11 = r_a
    err = np.abs(m.mask[:k_a] - 1.0).max()
    expect = np.array([c ** 0.125 for c in _COS_K_PI_12])
    return max(err, np.abs(m.mask[k_a:] - expect).max())


def test_absorber_mask_values():
    """The mask is 1 below r_max - 2 and cos(pi (r - r_a)/4)^(1/8) above:
    e.g. 2^(-1/16) halfway in, 2^(-1/8) two thirds in."""
    m = _mask_model()
    assert _mask_error(m) < 1e-15
    np.testing.assert_allclose(m.mask[33], 2.0 ** (-1.0 / 16.0), rtol=1e-15)
    np.testing.assert_allclose(m.mask[34], 2.0 ** (-1.0 / 8.0), rtol=1e-15)


def test_absorber_removed_norm_of_flat_density():
    """One absorber pass over a density rho = 1 removes sum (1 - m^2) dr.
    With r_a on the grid this left Riemann sum of 1 - cos^(1/4) equals
    w - (w/sqrt(pi)) Gamma(5/8)/Gamma(9/8) - dr/2 (w = 2 a0; the integral of
    cos^(1/4) over a quarter period by the Beta function, less the
    Euler-Maclaurin end term) up to O(dr^(5/4)) from the (w - x)^(1/4)
    behaviour at r_max: the residual shrinks by 4^(5/4) = 5.7 when dr
    falls 4-fold (measured 4.4e-4 -> 7.8e-5)."""
    w = 2.0
    exact = w - (w / math.sqrt(math.pi)) * gamma(5.0 / 8.0) / gamma(9.0 / 8.0)
    errs = []
    for n_r in (6144, 24576):        # r_a = 11 is grid point 5 n_r / 6
        dr = 12.0 / n_r
        m = MoleculeModel(n_r, 1.0, 13.0, 0, MASS, DT, np.zeros(n_r), np.zeros(n_r),
                          np.zeros(n_r), absorb_width=w)
        psi = np.ones((1, 2, 1, n_r), complex) / math.sqrt(2.0)      # |psi|^2 summed over s = 1
        _, lost = m.absorb(psi, np.zeros(1))
        errs.append(abs(lost[0] - (exact - dr / 2.0)) / exact)
    assert errs[0] < 1e-3 and errs[1] < 2e-4, errs
    assert 4.5 < errs[0] / errs[1] < 7.0, errs


@pytest.mark.parametrize("exponent", [8.0, 0.25, 0.5])
def test_absorber_pin_catches_planted_exponent(exponent):
    assert _mask_error(_mask_model(exponent=exponent)) > 1e-2


def test_absorber_pin_catches_planted_width():
    """r_a = r_max - w/2 instead of r_max - w."""
    n_r = 36
    m = MoleculeModel(n_r, 1.0, 13.0, 1, MASS, DT, np.zeros(n_r), np.zeros(n_r), np.zeros(n_r),
                      absorb_width=1.0)
    assert _mask_error(m) > 1e-2


# ---------------------------------------------------------------- Morse v = 0
def _fgh_ground(cfg):
    """Lowest eigenpair of the Fourier-grid Hamiltonian of U_g on the
    workload's periodic radial grid: the kinetic matrix is F^H diag(k^2/2mu) F
    / N with F the DFT matrix, the potential diagonal."""
    n = cfg.n_r
    dr = (cfg.r_max - cfg.r_min) / n
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    ms = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    k = 2.0 * np.pi * ms / (n * dr)
    H = (np.conj(F).T @ np.diag(k * k / (2.0 * cfg.mass)) @ F / n).real
    ug, _, _ = potentials(cfg)
    H += np.diag(ug)
    w, V = np.linalg.eigh(H)
    v = V[:, 0] / math.sqrt(dr)
    v *= np.sign(v[np.argmax(np.abs(v))])
    return w[0], v, H, dr


def _morse_e0(cfg):
    we = cfg.morse_a * math.sqrt(2.0 * cfg.morse_d / cfg.mass)
    return 0.5 * we - (0.5 * we) ** 2 / (4.0 * cfg.morse_d)


def _v0_errors(cfg, psi):
    e0, v, H, dr = _fgh_ground(cfg)
    vec = np.abs(psi - v).max() / np.abs(v).max()
    energy = abs(psi @ H @ psi * dr - _morse_e0(cfg)) / _morse_e0(cfg)
    return vec, energy, abs(e0 - _morse_e0(cfg)) / _morse_e0(cfg)


@pytest.mark.parametrize("name,vec_tol,e_tol", [("cfg0", 2e-6, 1e-8), ("cfg1", 1e-12, 1e-13)])
def test_morse_v0_is_the_grid_ground_state(name, vec_tol, e_tol):
    """The closed-form v = 0 function sampled on the grid equals the lowest
    eigenvector of the grid Hamiltonian (N_r = 128: 7.1e-7 of the peak, the
    grid's own truncation; N_r = 256: about 1e-14), its energy equals
    w_e/2 - w_e^2/(16 D), and it is discretely normalised."""
    cfg = get_config(name)
    psi = morse_v0(cfg)
    vec, energy, grid_e0 = _v0_errors(cfg, psi)
    assert vec < vec_tol, vec
    assert energy < e_tol and grid_e0 < e_tol, (energy, grid_e0)
    dr = (cfg.r_max - cfg.r_min) / cfg.n_r
    assert abs(np.sum(psi * psi) * dr - 1.0) < 1e-14


@pytest.mark.parametrize("dlam", [0.5, -0.5])
def test_morse_v0_pin_catches_lambda_slip(dlam):
    """A start with lambda -> lambda +- 1/2 (the exponent (lambda - 1/2) read
    as lambda, or the reverse) fails the pin: the function is built from a
    mass that shifts lambda = sqrt(2 mu D)/a by dlam, and compared with the
    true workload's grid ground state."""
    cfg = get_config("cfg1")
    lam = math.sqrt(2.0 * cfg.mass * cfg.morse_d) / cfg.morse_a
    mass = ((lam + dlam) * cfg.morse_a) ** 2 / (2.0 * cfg.morse_d)
    psi = morse_v0(cfg.replace(mass=mass))
    vec, energy, _ = _v0_errors(cfg, psi)
    assert vec > 1e-3 and energy > 1e-5, (vec, energy)      # measured 2.7e-3, 3.7e-5
