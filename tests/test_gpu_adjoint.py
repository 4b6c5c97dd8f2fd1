"""GPU checks of the hand-written adjoint of the coupled step.

1. One reverse step against the forward: <lambda', J delta> (central
   differences of the forward step) equals <J^T lambda', delta> (adjoint_step)
   for random state perturbations and adjoints, all state components at once
   (wavepackets, absorbed norms, cell polarisation, E, H, Drude currents, CPML
   auxiliaries) plus the source sample; FP64, tolerance 1e-7 relative.
2. The gradient of the dissociated population of a whole checkpointed run
   along a random direction of (64 knots, carrier) against the FP64 oracle's
   tangent-linear derivative (1e-8 relative in the FP64 form, 1e-3 in FP32).
3. The same gradient against central finite differences of the FP64 GPU
   form with a relative step of 1e-4 (tolerance 1e-3).
"""

import numpy as np
import pytest
import torch

from gpu_helpers import banner
from oracle.tangent import CoupledTangent, source_derivatives
from workloads import get_config
from workloads.geometry import material_map
from workloads.pulses import knot_values, source_values

pytestmark = pytest.mark.gpu


def _cfg(n_steps=120, j_max=6):
    return get_config("cfg0", n_r=128, j_max=j_max, pulse="knots", n_knots=64, knot_seed=4,
                      n_steps=n_steps, omega_h=0.10, ckpt_every=40)


def _cfg_dissociating(n_steps=250, ckpt=80):
    """A regime where the yield is a real signal: carrier near the vertical
    gap (one-photon excitation), lighter nuclei and r_diss = 4 a0, so the
    excited packet crosses r_diss within the run and Y is far above the FP32
    round-off floor (with the 0.10 Eh carrier and 120 steps of the tiny case
    Y ~ 1e-12, which FP32 cannot resolve and finite differences cannot
    difference)."""
    return get_config("cfg0", n_r=128, j_max=6, mass=500.0, r_diss=4.0, pulse="knots", n_knots=64,
                      knot_seed=4, n_steps=n_steps, omega_h=0.45, ckpt_every=ckpt)


def _mat_with_metal(cfg):
    mat = material_map(cfg)
    mat[:, 15:17] = 2      # a Drude layer above the molecules
    mat[:, 19:] = 1        # glass into the top CPML
    return mat


STATE = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "JDx", "JDy", "JDz", "psi"]


def _dot_state(sysm, vec):
    """<vec, state> over the differentiable state (real inner product)."""
    s = 0.0
    for k in STATE:
        s += float((vec[k] * sysm.fields.t[k]).sum())
    s += float((torch.conj(vec["mol_psi"]) * sysm.mol.psi).real.sum())
    s += float((vec["absorbed"] * sysm.mol.absorbed).sum())
    s += float((vec["P_c"] * sysm.P_c).sum())
    return s


@pytest.mark.parametrize("next_state,j_max,n_mol", [(False, 6, None), (True, 6, None), (True, 10, None),
                                                    (False, 6, 0)])
def test_adjoint_step_dot_product_fp64(next_state, j_max, n_mol):
    """With next_state the forward step is taken out of place (coupled_step's
    psi_next), which must equal the in-place step bit for bit and leave its
    input untouched, and the reverse step reads the state after the step
    (adjoint_step's psi_np1) instead of recomputing it.  j_max = 6 (N_J = 7)
    takes the half-K contractions, j_max = 10 all four K instructions.
    n_mol = 0: the fields alone (the source gradient's launch without the
    deposit's transpose, the H transpose without the gather's)."""
    from paper_2209_04487_amd import msqd
    cfg = _cfg(j_max=j_max)
    if n_mol is not None:
        cfg = cfg.replace(n_mol=n_mol)
    banner(f"adjoint step dot product fp64, j_max {j_max}, {cfg.n_mol} molecules, state after the step "
           f"{'given' if next_state else 'recomputed'}")
    mat = _mat_with_metal(cfg)
    kn = knot_values(cfg) * 30.0
    src = source_values(cfg, 0, 60, knots=kn)
    sysm = msqd.Coupled(cfg, prec="fp64", mat=mat,
                        cells=np.zeros(0, np.int32) if cfg.n_mol == 0 else None)
    if cfg.n_mol == 0:
        assert sysm.desc.n_occ == 0
    sysm.step(src[:40])
    x = sysm.snapshot()
    gen = torch.Generator(device="cpu").manual_seed(0)

    def rnd_like(t, scale):
        if t.is_complex():
            r = torch.randn(t.shape, generator=gen, dtype=torch.float64) + 1j * torch.randn(
                t.shape, generator=gen, dtype=torch.float64)
            return (r * scale).to(t.dtype).to(t.device)
        return (torch.randn(t.shape, generator=gen, dtype=torch.float64) * scale).to(t.dtype).to(t.device)

    def scale_of(t):
        v = float(t.abs().max()) if t.numel() else 0.0
        return v if v > 0 else 1.0

    delta, lam = {}, {}
    for k in STATE:
        sc = scale_of(x[k]) if k != "psi" else scale_of(x["Ex"]) * 1e-3
        delta[k] = rnd_like(x[k], sc)
        lam[k] = rnd_like(x[k], 1.0 / sc)
    for k, t in [("mol_psi", x["mol_psi"]), ("absorbed", x["absorbed"]), ("P_c", x["P_c"])]:
        sc = scale_of(t)
        delta[k] = rnd_like(t, sc)
        lam[k] = rnd_like(t, 1.0 / sc)
    ds = float(abs(src[40]))

    def step_from(eps):
        sysm.restore(x)
        for k in STATE:
            sysm.fields.t[k].add_(eps * delta[k])
        sysm.mol.psi.add_(eps * delta["mol_psi"])
        sysm.mol.absorbed.add_(eps * delta["absorbed"])
        sysm.P_c.add_(eps * delta["P_c"])
        sysm.step(np.array([src[40] + eps * ds]))
        return _dot_state(sysm, lam)

    eps = 1e-6
    jv = (step_from(eps) - step_from(-eps)) / (2 * eps)

    # adjoint: restore x, recompute the step's gathered field, then reverse
    sysm.restore(x)
    psi_n = sysm.mol.psi.clone()
    psi_np1 = None
    if next_state:
        sysm.step(src[40:41])
        in_place = sysm.mol.psi.clone()
        sysm.restore(x)
        psi_np1 = torch.empty_like(psi_n)
        sysm.step_out_of_place(src[40], psi_n, psi_np1)
        assert torch.equal(psi_np1, in_place)
        assert torch.equal(sysm.mol.psi, psi_n)
    else:
        sysm.step(src[40:41])
    e_n = sysm.E_mol.clone()
    adj, buf = sysm.adjoint_buffers()
    for k in STATE:
        buf[k].copy_(lam[k])
    buf["lpsi"].copy_(lam["mol_psi"])
    buf["labs"][: lam["absorbed"].numel()].copy_(lam["absorbed"])
    buf["lP"][: lam["P_c"].numel()].copy_(lam["P_c"])
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    msqd.adjoint_step(sysm.desc, sysm.state, psi_n, e_n, adj, 40, g, psi_np1=psi_np1)
    torch.cuda.synchronize()
    jtl = 0.0
    for k in STATE:
        jtl += float((buf[k] * delta[k]).sum())
    jtl += float((torch.conj(buf["lpsi"]) * delta["mol_psi"]).real.sum())
    jtl += float((buf["labs"][: lam["absorbed"].numel()] * delta["absorbed"]).sum())
    jtl += float((buf["lP"][: lam["P_c"].numel()] * delta["P_c"]).sum())
    jtl += float(g[0]) * ds
    assert abs(jv - jtl) <= 1e-7 * max(abs(jv), abs(jtl)), (jv, jtl)


def _direction(cfg, seed=7):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(cfg.n_knots + 1)
    v[-1] *= cfg.omega * 1e-2
    return v


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
def test_gradient_matches_oracle_tangent(prec, tol):
    from paper_2209_04487_amd.grad import yield_and_gradient
    cfg = _cfg_dissociating()
    banner(f"adjoint gradient vs oracle tangent {prec}")
    kn = knot_values(cfg) * 10.0
    Y, dk, dw = yield_and_gradient(cfg, kn, cfg.omega, prec=prec)
    v = _direction(cfg)
    dY_gpu = float(dk @ v[:-1] + dw * v[-1])
    tl = CoupledTangent(cfg)
    dsrc = v @ source_derivatives(cfg, cfg.n_steps, knots=kn)
    Y_o, dY_o = tl.run(source_values(cfg, 0, cfg.n_steps, knots=kn), dsrc)
    print(f"{prec}: Y gpu {Y:.12e} oracle {Y_o:.12e}; dY gpu {dY_gpu:.12e} oracle {dY_o:.12e}")
    assert Y_o > 5e-5          # a real dissociation signal
    assert abs(Y - Y_o) <= (1e-10 if prec == "fp64" else 1e-4) * abs(Y_o)
    assert abs(dY_gpu - dY_o) <= tol * abs(dY_o)


def test_gradient_matches_central_differences():
    from paper_2209_04487_amd.grad import CoupledYield, yield_and_gradient
    cfg = _cfg_dissociating(n_steps=200, ckpt=70)
    banner("adjoint gradient vs GPU central differences fp64")
    kn = knot_values(cfg) * 10.0
    Y, dk, dw = yield_and_gradient(cfg, kn, cfg.omega, prec="fp64")

    def Yof(knots, omega):
        k = torch.as_tensor(knots)
        w = torch.as_tensor(float(omega), dtype=torch.float64)
        return float(CoupledYield.apply(k, w, cfg, "fp64", None))

    for j in [int(np.argmax(np.abs(dk))), 20, 35]:
        h = 1e-4 * kn[j]
        kp, km = kn.copy(), kn.copy()
        kp[j] += h
        km[j] -= h
        fd = (Yof(kp, cfg.omega) - Yof(km, cfg.omega)) / (2 * h)
        assert abs(fd - dk[j]) <= 1e-3 * abs(dk[j]), (j, fd, dk[j])
    h = 1e-4 * cfg.omega
    fd = (Yof(kn, cfg.omega + h) - Yof(kn, cfg.omega - h)) / (2 * h)
    assert abs(fd - dw) <= 1e-3 * abs(dw), (fd, dw)


def test_full_size_gradient_fp64_fd_and_fp32():
    """The differentiation workload at its full size and launch shape (one
    SRR cell 96 x 96 x 80, 20,000 molecules, N_r = 128, J <= 6, a checkpoint
    every 200 steps) in the dissociating regime (lighter nuclei, carrier at
    the vertical gap, r_diss = 4 a0, 600 steps, so that the yield, about
    3e-5, is far above the FP32 round-off floor): the FP64 gradient against
    central differences of the FP64 forward (relative step 1e-4) on two knots
    and the carrier, and the FP32 yield and gradient against FP64, each to
    1e-3."""
    from paper_2209_04487_amd.grad import CoupledYield, yield_and_gradient
    cfg = get_config("cfg3", mass=500.0, r_diss=4.0, omega_h=0.45, n_steps=600, ckpt_every=200)
    banner(f"full-size adjoint cfg3: {cfg.n_mol} molecules, {cfg.nx}x{cfg.ny}x{cfg.nz}, {cfg.n_steps} steps")
    kn = knot_values(cfg) * 10.0
    Y, dk, dw = yield_and_gradient(cfg, kn, cfg.omega, prec="fp64")
    assert Y > 1e-6

    def Yof(knots, omega):
        k = torch.as_tensor(knots)
        w = torch.as_tensor(float(omega), dtype=torch.float64)
        return float(CoupledYield.apply(k, w, cfg, "fp64", None))

    for j in [int(np.argmax(np.abs(dk))), 20]:
        h = 1e-4 * kn[j]
        kp, km = kn.copy(), kn.copy()
        kp[j] += h
        km[j] -= h
        fd = (Yof(kp, cfg.omega) - Yof(km, cfg.omega)) / (2 * h)
        assert abs(fd - dk[j]) <= 1e-3 * abs(dk[j]), (j, fd, dk[j])
    h = 1e-4 * cfg.omega
    fd = (Yof(kn, cfg.omega + h) - Yof(kn, cfg.omega - h)) / (2 * h)
    assert abs(fd - dw) <= 1e-3 * abs(dw), (fd, dw)
    Y32, dk32, dw32 = yield_and_gradient(cfg, kn, cfg.omega, prec="fp32")
    assert abs(Y32 - Y) <= 1e-3 * abs(Y)
    assert np.abs(dk32 - dk).max() <= 1e-3 * np.abs(dk).max()
    assert abs(dw32 - dw) <= 1e-3 * abs(dw)


def test_multirate_gradient_matches_central_differences():
    """Multi-rate coupling (molecules by 4 dt every 4 field steps, the current
    held in between): the FP64 gradient against central differences of the
    FP64 forward on two knots and the carrier, and FP32 against FP64, each
    to 1e-3, over 250 steps (Y ~ 1e-4).  Checkpoints every 70 steps, so that
    segments restart in the middle of a held interval."""
    from paper_2209_04487_amd.grad import CoupledYield, yield_and_gradient
    M = 4
    cfg = _cfg_dissociating(n_steps=250, ckpt=70)
    banner(f"adjoint gradient multi-rate M={M} vs GPU central differences fp64")
    kn = knot_values(cfg) * 10.0
    Y, dk, dw = yield_and_gradient(cfg, kn, cfg.omega, prec="fp64", mol_every=M)
    assert Y > 1e-5

    def Yof(knots, omega):
        k = torch.as_tensor(knots)
        w = torch.as_tensor(float(omega), dtype=torch.float64)
        return float(CoupledYield.apply(k, w, cfg, "fp64", None, M))

    for j in [int(np.argmax(np.abs(dk))), 20]:
        h = 1e-4 * kn[j]
        kp, km = kn.copy(), kn.copy()
        kp[j] += h
        km[j] -= h
        fd = (Yof(kp, cfg.omega) - Yof(km, cfg.omega)) / (2 * h)
        assert abs(fd - dk[j]) <= 1e-3 * abs(dk[j]), (j, fd, dk[j])
    h = 1e-4 * cfg.omega
    fd = (Yof(kn, cfg.omega + h) - Yof(kn, cfg.omega - h)) / (2 * h)
    assert abs(fd - dw) <= 1e-3 * abs(dw), (fd, dw)
    Y32, dk32, dw32 = yield_and_gradient(cfg, kn, cfg.omega, prec="fp32", mol_every=M)
    assert abs(Y32 - Y) <= 1e-3 * abs(Y)
    assert np.abs(dk32 - dk).max() <= 1e-3 * np.abs(dk).max()
    assert abs(dw32 - dw) <= 1e-3 * abs(dw)
