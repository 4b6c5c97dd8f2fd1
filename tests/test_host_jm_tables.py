"""Host logic of the general (j, m) coupling (no device): the tables that
qd_init places in the workspace, read through qd_jm_tables, against the
oracle's direction-cosine matrices (product quadrature of the spherical
harmonics).  The rotation U = exp(-i alpha J_z) exp(-i beta J_y), with
d^j(beta) formed from the J_x eigenvectors, and the per-m' eigenvectors Q of
cos(theta) must diagonalise A(E) = sum_c E_c D_c for any field, with
eigenvalues |E| x_k; the dipole matrix elements must equal the oracle's."""

import numpy as np
import pytest

from oracle.molecule_jm import direction_cosines, jm_basis


def _layout(jm):
    off = lambda j: j * (4 * j * j - 1) // 3
    sq = lambda n: n * (n + 1) * (2 * n + 1) // 6
    qoff = lambda a: sq(jm + 1) - sq(jm + 1 - a)
    xoff = lambda a: a * (jm + 1) - a * (a - 1) // 2
    return off, qoff, xoff, off(jm + 1), qoff(jm + 1), xoff(jm + 1)


def _rotation(v, jm, E):
    off, _, _, _, _, _ = _layout(jm)
    basis = jm_basis(jm)
    idx = {b: i for i, b in enumerate(basis)}
    e = np.linalg.norm(E)
    rho = np.hypot(E[0], E[1])
    ea = (E[0] + 1j * E[1]) / rho if rho > 0 else 1.0
    beta = np.arctan2(rho, E[2])
    U = np.zeros((len(basis), len(basis)), complex)
    for j in range(jm + 1):
        n = 2 * j + 1
        O = v[off(j):off(j) + n * n].reshape(n, n)
        mu = np.arange(n) - j
        for a in range(n):
            for c in range(n):
                ang = 0.5 * np.pi * (c - a) - beta * mu
                d = np.sum(O[a] * O[c] * np.cos(ang))
                U[idx[(j, a - j)], idx[(j, c - j)]] = ea ** (-(a - j)) * d
    return U, e, idx


@pytest.mark.parametrize("jm", [2, 3, 4, 5])
def test_tables_diagonalise_the_coupling(msqd, jm):
    v = msqd.jm_tables(jm)
    off, qoff, xoff, n_jx, n_q, n_x = _layout(jm)
    assert len(v) == n_jx + n_q + n_x + 3 * (jm + 1) ** 2
    D = direction_cosines(jm)
    nb = (jm + 1) ** 2
    rng = np.random.default_rng(jm)
    fields = [rng.normal(size=3) for _ in range(3)] + [np.array([0.0, 0.0, -0.7]), np.array([0.4, 0.0, 0.0])]
    for E in fields:
        U, e, idx = _rotation(v, jm, E)
        W = np.zeros((nb, nb), complex)
        lam = np.zeros(nb)
        col = 0
        for mp in range(-jm, jm + 1):
            a = abs(mp)
            n = jm + 1 - a
            Q = v[n_jx + qoff(a):n_jx + qoff(a) + n * n].reshape(n, n)
            x = v[n_jx + n_q + xoff(a):n_jx + n_q + xoff(a) + n]
            assert np.all(np.diff(x) > 0)
            for k in range(n):
                W[:, col] = sum(Q[i, k] * U[:, idx[(a + i, mp)]] for i in range(n))
                lam[col] = e * x[k]
                col += 1
        A = np.einsum("c,cab->ab", E, D)
        assert np.abs(W.conj().T @ W - np.eye(nb)).max() < 1e-13
        assert np.abs(A @ W - W * lam).max() < 1e-13 * max(e, 1.0)
        assert np.allclose(np.sort(lam), np.linalg.eigvalsh(A), atol=1e-13)


@pytest.mark.parametrize("jm", [2, 5])
def test_dipole_matrix_elements(msqd, jm):
    v = msqd.jm_tables(jm)
    _, _, _, n_jx, n_q, n_x = _layout(jm)
    D = direction_cosines(jm)
    idx = {b: i for i, b in enumerate(jm_basis(jm))}
    dip = v[n_jx + n_q + n_x:].reshape(-1, 3)
    Dp = D[0] + 1j * D[1]
    for (j, m), b in idx.items():
        z = D[2][idx[(j + 1, m)], b] if j < jm else 0.0
        up = Dp[idx[(j + 1, m + 1)], b] if j < jm else 0.0
        dn = Dp[idx[(j - 1, m + 1)], b] if m + 1 <= j - 1 else 0.0
        np.testing.assert_allclose(dip[b], [z, np.real(up), np.real(dn)], atol=1e-13)
        # the elements are real (Condon-Shortley phases)
        assert abs(np.imag(up)) < 1e-13 and abs(np.imag(dn)) < 1e-13


def test_tables_reject_bad_arguments(msqd):
    import ctypes as C
    assert msqd.lib.qd_jm_tables_size(1) == 0 and msqd.lib.qd_jm_tables_size(6) == 0
    out = np.zeros(10)
    p = out.ctypes.data_as(C.POINTER(C.c_double))
    assert msqd.lib.qd_jm_tables(1, p, 10) == msqd.MSQD_EUNSUP
    assert msqd.lib.qd_jm_tables(2, p, 10) == msqd.MSQD_ESHAPE
    assert msqd.lib.qd_jm_tables(2, None, 100) == msqd.MSQD_EINVAL


@pytest.fixture(scope="module")
def msqd():
    from paper_2209_04487_amd import msqd as m
    return m
