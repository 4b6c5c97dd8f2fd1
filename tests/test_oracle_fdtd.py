"""Pins of the oracle's Yee/Drude/CPML update against closed forms.

- the exact discrete dispersion of the Yee scheme (an eigenmode of a fully
  periodic vacuum box advances by exactly exp(-i omega_d dt) per step),
- the continuum Drude plasma oscillation (second-order convergence),
- Fresnel transmission 4n/(1+n)^2 of a vacuum/glass interface at normal
  incidence, with the soft source's incident amplitude and the monitor's
  plane-wave flux |E|^2 / (2 eta0),
- CPML: the field energy left in an open 1-D run after the pulse has gone.
"""

import math

import numpy as np
import pytest

from oracle.fdtd import C0, EPS0, ETA0, MU0, FluxMonitor, Yee

# positions (cell units) of the six field components
E_POS = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))
H_POS = ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def _phase(shape, K, pos, dx):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) + pos[2], np.arange(ny) + pos[1],
                          np.arange(nx) + pos[0], indexing="ij")
    return np.exp(1j * (K[0] * x + K[1] * y + K[2] * z) * dx)


@pytest.mark.parametrize("n", [(1, 2, 3), (3, 0, 1), (0, 0, 2)])
def test_yee_vacuum_eigenmode_exact_dispersion(n):
    nx, ny, nz = 8, 6, 10
    dx = 3e-9
    dt = 0.5 * dx / C0
    shape = (nz, ny, nx)
    K = 2 * np.pi * np.array([n[0] / (nx * dx), n[1] / (ny * dx), n[2] / (nz * dx)])
    Kt = 2.0 / dx * np.sin(K * dx / 2)
    # polarisation perpendicular to the discrete wave vector
    a = np.cross(Kt, np.array([0.3, -0.7, 0.2]))
    Ehat = a / np.linalg.norm(a)
    w = 2.0 / dt * math.asin(C0 * dt * np.linalg.norm(Kt) / 2)
    Hhat = dt / (2 * MU0 * math.sin(w * dt / 2)) * np.cross(Kt, Ehat)
    mat = np.zeros((3,) + shape, np.uint8)
    yee = Yee(nx, ny, nz, dx, dt, mat, [1.0, 1.0, 1.0], 0.0, 0.0, 0, periodic_z=True)
    for c in range(3):
        yee.E[c][:] = (Ehat[c] * _phase(shape, K, E_POS[c], dx)).real
        yee.H[c][:] = (Hhat[c] * _phase(shape, K, H_POS[c], dx) * np.exp(1j * w * dt / 2)).real
    nsteps = 300
    for _ in range(nsteps):
        yee.update_H()
        yee.update_E()
    for c in range(3):
        expect = (Ehat[c] * _phase(shape, K, E_POS[c], dx) * np.exp(-1j * w * nsteps * dt)).real
        np.testing.assert_allclose(yee.E[c], expect, atol=1e-11)


def _drude_run(dt, wp, gamma, eps_inf, t_end, E0=1.0):
    mat = np.full((3, 1, 1, 1), 2, np.uint8)
    yee = Yee(1, 1, 1, 1e-9, dt, mat, [1.0, 2.25, eps_inf], wp, gamma, 0, periodic_z=True)
    wd = math.sqrt(wp * wp / eps_inf - gamma * gamma / 4)

    def exact(t):
        return E0 * math.exp(-gamma * t / 2) * (math.cos(wd * t) + gamma / (2 * wd) * math.sin(wd * t))

    def current(t):
        return EPS0 * eps_inf * E0 * math.exp(-gamma * t / 2) * (wd + gamma ** 2 / (4 * wd)) * math.sin(wd * t)

    yee.E[0][:] = E0
    yee.JD[0][:] = current(-dt / 2)
    n = int(round(t_end / dt))
    err = 0.0
    for s in range(1, n + 1):
        yee.update_H()
        yee.update_E()
        err = max(err, abs(yee.E[0][0, 0, 0] - exact(s * dt)))
    return err / E0


def test_drude_plasma_oscillation_second_order():
    """Uniform E in a periodic metal box: eps0 eps_inf dE/dt = -J and
    dJ/dt + gamma J = eps0 wp^2 E give E'' + gamma E' + (wp^2/eps_inf) E = 0;
    the centred discretisation converges to it at second order."""
    wp = 9.1 / 6.582119569e-16
    gamma = 0.5 / 6.582119569e-16          # large damping to test that term too
    eps_inf = 3.7
    period = 2 * math.pi / math.sqrt(wp * wp / eps_inf)
    dt = period / 200
    e1 = _drude_run(dt, wp, gamma, eps_inf, 3 * period)
    e2 = _drude_run(dt / 2, wp, gamma, eps_inf, 3 * period)
    assert e1 < 2e-3
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def _run_1d(glass_from, nsteps, nz=300, dx=5e-9, npml=20, src_k=40, mon_k=220,
            omegas=None, record_energy=False):
    dt = 0.5 * dx / C0
    mat = np.zeros((3, nz, 1, 1), np.uint8)
    if glass_from is not None:
        for c in range(3):
            zc = np.arange(nz) + (0.5 if c == 2 else 0.0)
            mat[c][zc >= glass_from] = 1
    eps_hi = 2.25 if glass_from is not None else 1.0
    smax = lambda e: 0.8 * 4 / (ETA0 * dx * math.sqrt(e))  # noqa: E731
    yee = Yee(1, 1, nz, dx, dt, mat, [1.0, 2.25, 1.0], 0.0, 0.0, npml, 3.0,
              smax(1.0), smax(eps_hi))
    mon = FluxMonitor(1, 1, mon_k, omegas, dt, 1)
    mon2 = FluxMonitor(1, 1, 100, omegas, dt, 1)
    tau = 1.0e-15
    t0 = 3.0e-15
    w0 = 0.10 / 2.4188843265857e-17
    src = []
    energy = []
    for n in range(nsteps):
        t = (n + 0.5) * dt
        v = math.exp(-4 * math.log(2) * (t - t0) ** 2 / tau ** 2) * math.cos(w0 * (t - t0))
        src.append(v)
        yee.update_H()
        yee.update_E(v, src_k)
        mon.sample(yee, n)
        mon2.sample(yee, n)
        if record_energy:
            energy.append(yee.energy())
    _run_1d.mon2 = mon2
    return yee, mon, np.array(src), dt, np.array(energy)


def test_fresnel_transmission_and_source_amplitude():
    omegas = np.array([0.08, 0.09, 0.10, 0.11, 0.12]) / 2.4188843265857e-17
    nsteps = 1500
    _, mon_v, src, dt, _ = _run_1d(None, nsteps, omegas=omegas)
    _, mon_g, _, _, _ = _run_1d(150, nsteps, omegas=omegas)
    T = mon_g.flux() / mon_v.flux()
    n = 1.5
    np.testing.assert_allclose(T, 4 * n / (1 + n) ** 2, atol=2e-3)
    # incident plane wave: amplitude equal to E_inc, flux |E|^2 / (2 eta0)
    t = (np.arange(nsteps) + 0.5) * dt
    S = np.array([np.sum(src * np.exp(1j * w * t)) * dt for w in omegas])
    Ex = mon_v.Ex[:, 0, 0]
    np.testing.assert_allclose(np.abs(Ex) / np.abs(S), 1.0, atol=1e-2)
    np.testing.assert_allclose(mon_v.flux(), np.abs(Ex) ** 2 / (2 * ETA0), rtol=1e-2)


def test_cpml_absorbs_outgoing_pulse():
    omegas = np.array([0.1]) / 2.4188843265857e-17
    _, _, _, _, energy = _run_1d(None, 2400, omegas=omegas, record_energy=True)
    assert energy[-1] / energy.max() < 1e-6


def test_reflection_and_absorption_spectra_of_a_dielectric_interface():
    """Two detection planes (incident side and transmitted side) and a
    vacuum reference run: a lossless glass interface reflects
    ((n-1)/(n+1))^2, transmits 4n/(n+1)^2 and absorbs nothing."""
    from oracle.fdtd import spectra
    omegas = np.array([0.08, 0.10, 0.12]) / 2.4188843265857e-17
    nsteps = 1500
    _, mon_v, _, _, _ = _run_1d(None, nsteps, omegas=omegas)
    ref2 = _run_1d.mon2.flux()
    _, mon_g, _, _, _ = _run_1d(150, nsteps, omegas=omegas)
    inc2 = _run_1d.mon2.flux()
    T, R, A = spectra(mon_g.flux(), inc2, ref2)
    n = 1.5
    np.testing.assert_allclose(R, ((n - 1) / (n + 1)) ** 2, atol=2e-3)
    np.testing.assert_allclose(T, 4 * n / (1 + n) ** 2, atol=2e-3)
    np.testing.assert_allclose(A, 0.0, atol=3e-3)
