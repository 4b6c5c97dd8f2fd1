"""Pins of the Bloch-emitter oracle (frozen two-level molecules, RK4):

- a static field has the closed-form detuned Rabi solution
  P_e(t) = (4V^2/W^2) sin^2(W t / 2), W = sqrt(w0^2 + 4V^2), V = -mu E;
- the integrator is fourth order (error ratio 16 when dt halves);
- without relaxation the Bloch vector keeps unit length;
- with relaxation and no field, rho_ee decays as exp(-g1 t) and rho_ge turns
  at w0 while decaying as exp(-g2 t);
- coupled to the grid, the field energy lost equals the emitters' energy
  w0 rho_ee gained, to first order in dt (fixes the current's sign and units).
"""

import numpy as np

from oracle.bloch import BlochModel, CoupledBlochOracle
from oracle.fdtd import EPS0, Yee
from workloads import get_config

EH_J = 4.3597447222071e-18


def _rabi(model, E, t):
    V = -model.mu * E
    W = np.sqrt(model.w0 ** 2 + 4 * V ** 2)
    return 4 * V ** 2 / W ** 2 * np.sin(W * t / 2) ** 2


def _run(model, E, nsteps, y=None):
    y = BlochModel.ground(len(E)) if y is None else y
    for _ in range(nsteps):
        y = model.step(y, E)
    return y


def test_static_field_detuned_rabi():
    E = np.array([0.02, -0.05, 0.1])
    m = BlochModel(0.3, 1.2, 0.01)
    y = _run(m, E, 2000)
    np.testing.assert_allclose(y[0], _rabi(m, E, 20.0), atol=1e-9)


def test_fourth_order():
    E = np.array([0.08])
    errs = []
    for dt in (0.2, 0.1, 0.05):
        m = BlochModel(0.4, 1.0, dt)
        y = _run(m, E, int(round(10.0 / dt)))
        errs.append(abs(y[0, 0] - _rabi(m, E, 10.0)[0]))
    assert 13.0 < errs[0] / errs[1] < 19.0, errs
    assert 13.0 < errs[1] / errs[2] < 19.0, errs


def test_bloch_vector_length_conserved():
    rng = np.random.default_rng(1)
    E = rng.uniform(-0.1, 0.1, 16)
    m = BlochModel(0.47, 0.6, 0.02)
    y = _run(m, E, 3000)
    length = (2 * y[0] - 1) ** 2 + 4 * (y[1] ** 2 + y[2] ** 2)
    np.testing.assert_allclose(length, 1.0, atol=1e-8)


def test_free_relaxation():
    g1, g2, w0, dt, n = 0.01, 0.03, 0.5, 0.02, 5000
    m = BlochModel(w0, 1.0, dt, gamma1=g1, gamma2=g2)
    y = np.array([[0.5], [0.5], [0.0]])
    y = _run(m, np.zeros(1), n, y)
    t = n * dt
    np.testing.assert_allclose(y[0, 0], 0.5 * np.exp(-g1 * t), rtol=1e-9)
    rho = 0.5 * np.exp((1j * w0 - g2) * t)
    np.testing.assert_allclose(y[1, 0] + 1j * y[2, 0], rho, atol=1e-10)


def _closed_box(courant):
    cfg = get_config("cfg0", nx=2, ny=2, nz=2, courant=courant, mol_weight=1e4,
                     n_mol=8, placement="block", block_lo=0, block_n=2, mon_k=1)
    mat = np.zeros((3, 2, 2, 2), np.uint8)
    yee = Yee(2, 2, 2, cfg.dx, cfg.dt, mat, [1, 1, 1], 0.0, 0.0, 0, periodic_z=True)
    model = BlochModel(0.05, 1.0, cfg.dt_au)
    o = CoupledBlochOracle(cfg, model=model, mat=mat, yee=yee)
    yee.E[0][:] = 2e-3 * 5.14220674763e11
    return cfg, o, yee


def test_coupled_energy_balance_closed_box():
    imbalance = []
    for courant in (0.5, 0.25):
        cfg, o, yee = _closed_box(courant)
        f0 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
        nst = int(round(40 / courant))
        for n in range(nst):
            o.step(n, 0.0)
        f1 = np.sum(EPS0 * yee.E[0] ** 2 / 2) * cfg.dx ** 3
        m1 = cfg.mol_weight * np.sum(o.model.w0 * o.y[0]) * EH_J
        assert f1 < f0 and m1 > 0
        imbalance.append(((f1 + m1) - f0) / m1)
    assert abs(imbalance[0]) < 0.25, imbalance
    assert 1.6 < imbalance[0] / imbalance[1] < 2.4, imbalance
