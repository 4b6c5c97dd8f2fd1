"""Pins of the (j, m)-basis molecular oracle (all three field components):

- the direction-cosine matrices are Hermitian, d.d = 1 on j = 0 (the sum
  rule sum_c <00|D_c D_c|00> = 1) and D_z restricted to m = 0 is the m = 0
  model's cos(theta) matrix (closed-form c_J);
- with the field along z and only m = 0 components, one step equals the
  m = 0 oracle's step (whose angular DVR is pinned separately);
- isotropy: from the rotational ground state, a field along x, along y,
  along z or along (1, 1, 1)/sqrt(3) induces the same dipole along the field
  and none across it;
- the coupling factor equals a dense matrix exponential; without absorber the
  norm is conserved;
- rotational covariance: rotating the initial state (the rotation's matrix
  on each j block taken by quadrature of the spherical harmonics at rotated
  points, not from the direction cosines) and the field by the same rotation
  rotates the stepped state, and the dipole turns as a vector.
"""

import numpy as np
import pytest
from scipy.linalg import expm

from numpy.polynomial.legendre import leggauss
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

from oracle.molecule import MoleculeModel, coupling_cj
from oracle.molecule_jm import MoleculeJM, direction_cosines, jm_basis


def _models(j_max=1, n_r=64, dt=0.5, mass=1.0e4, absorb=0.0):
    r = 1.0 + 11.0 / n_r * np.arange(n_r)
    ug = 0.17 * (1 - np.exp(-(r - 2.0))) ** 2
    ue = 0.17 + 0.3 * np.exp(-1.2 * (r - 2.0))
    mu = np.exp(-0.1 * (r - 2.0) ** 2)
    jm = MoleculeJM(n_r, 1.0, 12.0, j_max, mass, dt, ug, ue, mu, absorb_width=absorb)
    m0 = MoleculeModel(n_r, 1.0, 12.0, j_max, mass, dt, ug, ue, mu, absorb_width=absorb)
    return jm, m0


@pytest.mark.parametrize("j_max", [1, 2, 3, 5])
def test_direction_cosine_matrices(j_max):
    D = direction_cosines(j_max)
    basis = jm_basis(j_max)
    for c in range(3):
        np.testing.assert_allclose(D[c], np.conj(D[c]).T, atol=1e-14)
    s = sum(D[c] @ D[c] for c in range(3))
    assert abs(s[0, 0] - 1.0) < 1e-13
    idx = [b for b, (j, m) in enumerate(basis) if m == 0]
    Dz0 = D[2][np.ix_(idx, idx)].real
    cj = coupling_cj(j_max)
    expect = np.diag(cj, 1) + np.diag(cj, -1)
    np.testing.assert_allclose(Dz0, expect, atol=1e-13)
    # selection rules: d_z keeps m, d_x and d_y change m by one
    for a, (j1, m1) in enumerate(basis):
        for b, (j2, m2) in enumerate(basis):
            if abs(D[2][a, b]) > 1e-13:
                assert m1 == m2 and abs(j1 - j2) == 1
            if abs(D[0][a, b]) > 1e-13 or abs(D[1][a, b]) > 1e-13:
                assert abs(m1 - m2) == 1 and abs(j1 - j2) == 1


@pytest.mark.parametrize("j_max", [1, 2])
def test_field_along_z_reduces_to_m0_model(j_max):
    jm, m0 = _models(j_max)
    rng = np.random.default_rng(j_max)
    psi0 = rng.standard_normal((2, 2, j_max + 1, jm.n_r)) + 1j * rng.standard_normal((2, 2, j_max + 1, jm.n_r))
    E = np.array([0.02, -0.05])
    p0, _ = m0.step(psi0, E, np.zeros(2))
    idx = [b for b, (j, m) in enumerate(jm.basis) if m == 0]
    full = np.zeros((2, 2, jm.n_b, jm.n_r), complex)
    full[:, :, idx] = psi0
    E3 = np.stack([np.zeros(2), np.zeros(2), E], axis=1)
    p1, _ = jm.step(full, E3, np.zeros(2))
    np.testing.assert_allclose(p1[:, :, idx], p0, atol=1e-12)
    other = [b for b in range(jm.n_b) if b not in idx]
    assert np.abs(p1[:, :, other]).max() < 1e-13
    np.testing.assert_allclose(jm.dipole(p1)[:, 2], m0.dipole(p0), rtol=1e-11)


def test_isotropy_of_the_induced_dipole():
    jm, _ = _models(j_max=2)
    r0 = np.exp(-((jm.r - 2.0) / 0.3) ** 2)
    r0 /= np.sqrt(np.sum(r0 ** 2) * jm.dr)
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    E3 = 0.05 * dirs
    psi = jm.initial_state(len(dirs), r0)
    ab = np.zeros(len(dirs))
    for _ in range(40):
        psi, ab = jm.step(psi, E3, ab)
    d = jm.dipole(psi)
    along = np.sum(d * dirs, axis=1)
    assert np.abs(along).max() > 1e-6
    np.testing.assert_allclose(along, along[2], rtol=1e-10)
    across = d - along[:, None] * dirs
    assert np.abs(across).max() < 1e-10 * np.abs(along).max()


@pytest.mark.parametrize("j_max,E", [(1, [0.03, -0.07, 0.05]), (3, [0.3, -0.2, 0.25]), (5, [-0.1, 0.4, -0.3])])
def test_coupling_is_the_dense_exponential_and_conserves_norm(j_max, E):
    jm, _ = _models(j_max=j_max, n_r=32)
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((1, 2, jm.n_b, jm.n_r)) + 1j * rng.standard_normal((1, 2, jm.n_b, jm.n_r))
    E3 = np.array([E])
    out = jm.coupling(psi, E3)
    A = np.einsum("c,cab->ab", E3[0], jm.D)
    sx = np.array([[0, 1], [1, 0]])
    for k in (0, 7, 31):
        U = expm(1j * jm.mu12[k] * jm.dt * np.kron(sx, A))
        np.testing.assert_allclose(out[0, :, :, k].reshape(-1), U @ psi[0, :, :, k].reshape(-1), atol=1e-12)
    p = psi.copy()
    ab = np.zeros(1)
    n0 = jm.norm(p)
    for _ in range(20):
        p, ab = jm.step(p, E3, ab)
    np.testing.assert_allclose(jm.norm(p), n0, rtol=1e-12)


def test_coupled_jm_energy_balance_with_transverse_field():
    """The coupled scheme in the (j, m) basis with the closed-box field along
    y (so only the E_y gather and J_y deposit act): the field energy lost
    equals the molecules' energy gained, to first order in dt, as for the
    m = 0 scheme along x."""
    from oracle.coupled import CoupledOracle
    from oracle.fdtd import EPS0, Yee
    from workloads import get_config
    EH_J = 4.3597447222071e-18
    imb = []
    for courant in (0.5, 0.25):
        cfg = get_config("cfg0", nx=2, ny=2, nz=2, courant=courant, mol_weight=1e4, n_mol=8,
                         placement="block", block_lo=0, block_n=2, mon_k=1, j_max=1, basis="jm",
                         n_r=64)
        mat = np.zeros((3, 2, 2, 2), np.uint8)
        yee = Yee(2, 2, 2, cfg.dx, cfg.dt, mat, [1, 1, 1], 0.0, 0.0, 0, periodic_z=True)
        o = CoupledOracle(cfg, mat=mat, yee=yee)
        yee.E[1][:] = 5e-2 * 5.14220674763e11
        m = o.mol

        def h0(psi):
            ph = np.fft.fft(psi, axis=-1)
            kin = np.sum(np.abs(ph) ** 2 * (m.kappa ** 2 / (2 * m.mass))[None, None, None, :],
                         axis=(1, 2, 3)) * m.dr / m.n_r
            jb = np.array([j for (j, _) in m.basis], float)
            V = m.U[:, None, :] + (jb * (jb + 1))[None, :, None] / (2 * m.mass * m.r[None, None, :] ** 2)
            return kin + np.sum(np.abs(psi) ** 2 * V[None], axis=(1, 2, 3)) * m.dr
        f0 = sum(np.sum(EPS0 * e ** 2 / 2) for e in yee.E) * cfg.dx ** 3
        m0 = cfg.mol_weight * np.sum(h0(o.psi)) * EH_J
        for n in range(int(round(100 / courant))):
            o.step(n, 0.0)
        f1 = sum(np.sum(EPS0 * e ** 2 / 2) for e in yee.E) * cfg.dx ** 3
        m1 = cfg.mol_weight * np.sum(h0(o.psi)) * EH_J
        assert f1 < f0 and m1 > m0
        assert np.abs(yee.E[0]).max() < 1e-6 * np.abs(yee.E[1]).max()
        imb.append(((f1 + m1) - (f0 + m0)) / (m1 - m0))
    assert abs(imb[0]) < 0.25, imb
    assert 1.6 < imb[0] / imb[1] < 2.4, imb


def _rotation_matrix_on_basis(j_max, R):
    """U[(j, m'), (j, m)] = int conj(Y_jm') (Y_jm o R^-1) dOmega by a product
    quadrature exact for these degrees: the action f -> f(R^-1 r) of the
    rotation R on the truncated basis."""
    basis = jm_basis(j_max)
    n_t = n_p = 2 * j_max + 4
    x, w = leggauss(n_t)
    th = np.arccos(x)
    ph = 2.0 * np.pi * np.arange(n_p) / n_p
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = w[:, None] * (2.0 * np.pi / n_p)
    pts = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1)
    back = pts @ R            # rows are R^T r = R^-1 r
    th2 = np.arccos(np.clip(back[..., 2], -1.0, 1.0))
    ph2 = np.arctan2(back[..., 1], back[..., 0])
    U = np.zeros((len(basis), len(basis)), complex)
    for a, (j1, m1) in enumerate(basis):
        y1 = np.conj(sph_harm_y(j1, m1, TH, PH))
        for b, (j2, m2) in enumerate(basis):
            if j1 == j2:
                U[a, b] = np.sum(W * y1 * sph_harm_y(j2, m2, th2, ph2))
    return U


@pytest.mark.parametrize("j_max", [1, 3])
def test_rotational_covariance(j_max):
    jm, _ = _models(j_max=j_max, n_r=32)
    rng = np.random.default_rng(11 + j_max)
    R = Rotation.random(random_state=rng.integers(1 << 31)).as_matrix()
    U = _rotation_matrix_on_basis(j_max, R)
    assert np.abs(U.conj().T @ U - np.eye(jm.n_b)).max() < 1e-12
    psi = rng.standard_normal((1, 2, jm.n_b, jm.n_r)) + 1j * rng.standard_normal((1, 2, jm.n_b, jm.n_r))
    E = np.array([[0.05, -0.08, 0.03]])
    p1, _ = jm.step(psi, E, np.zeros(1))
    psi_r = np.einsum("ab,msbr->msar", U, psi)
    p2, _ = jm.step(psi_r, E @ R.T, np.zeros(1))
    np.testing.assert_allclose(p2, np.einsum("ab,msbr->msar", U, p1), atol=1e-11)
    np.testing.assert_allclose(jm.dipole(p2)[0], R @ jm.dipole(p1)[0], atol=1e-11)
    # and a field that is not a rotation of the first one gives a different state
    p3, _ = jm.step(psi_r, E, np.zeros(1))
    assert np.abs(p3 - p2).max() > 1e-4
