"""Benchmark of the coupled Maxwell-Schroedinger step on one MI355X.

Workload: the silver split-ring-resonator array (192 x 192 x 120 Yee grid,
dx = 2 nm, Drude metal, glass substrate, CPML in z), 100,000 molecules in a
20 nm slab, radial grid N_r = 256, rotational basis J = 0..10, Gaussian pulse
(0.10 Eh carrier, FWHM 10 fs).  `value` is the throughput of the precision
form (complex64 wavepackets and FFTs, J<->angle transform on BF16 matrix
cores with a hi/lo split, FP32 fields, FP64 reductions) in molecule-steps/s
of the whole coupled step (H update, field gather, molecular step, per-cell
dipole reduction and polarisation current, E update with Drude and source,
flux monitor).  The plain FP64 form is timed on the same workload for the
comparison.

Accuracy: both forms are run from the same first step for --acc-steps steps
(default 1,000, covering the arrival of the pulse peak at the molecules),
recording the ensemble dipole after every step; the line reports the
relative L2 error of the precision form's dipole trace, of its transmitted
flux spectrum and of its mean dissociated population against the FP64 form.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions (not used by this
# library): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 78.6
# dense BF16 matrix-core peak (no structured sparsity)
BF16_MFMA_PEAK_TFLOPS = 2500.0
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "mol_step_mixed_srr100k_counters.md")
METRIC = "molecule-steps/s, coupled step, FP32/BF16 vs FP64 at ≤1e-4 rel dipole err"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mol_bytes_per_step(cfg, prec):
    """Algorithmic HBM bytes of one molecule-step: the wavepacket read and
    written once, plus the per-molecule field gather (value and cell index),
    the absorbed accumulator (read + write), the dipole and the recorded
    field."""
    el = 16 if prec == "fp64" else 8
    psi = 2 * cfg.n_j * cfg.n_r * el
    field = 8 if prec == "fp64" else 4
    return 2 * psi + field + 4 + 16 + 8 + 8


def mol_flops_per_step(cfg):
    """Algorithmic vector flops of one molecule-step: four N_r-point complex
    FFTs per (state, J) line (two kinetic half-steps, each a forward and an
    inverse transform; 5 N log2 N flops each), the kinetic and the two
    potential phase multiplies (6 flops per point each), the 2x2 coupling
    rotation at every (angle node, r) point (12 flops plus 2 for the angle),
    and the norm and dipole readouts.  The J<->angle contractions run on the
    matrix cores and are not counted here."""
    n, nj = cfg.n_r, cfg.n_j
    lines = 2 * nj
    fft = 5 * n * int(np.log2(n))
    per_line = 4 * fft + 2 * 6 * n + 2 * 6 * n
    rot = nj * n * 14
    readout = 2 * nj * n * 3 + (nj - 1) * n * 8
    return lines * per_line + rot + readout


def jm_flops_per_step(n_r):
    """Algorithmic vector flops of one molecule-step in the (j, m) basis with
    j <= 1 (four lines per state): four N_r-point complex FFTs per line, the
    kinetic and the two potential phase multiplies (6 flops per point each),
    and the closed-form coupling at every r: the two projections <v|g_1>,
    <v|e_1> (3 complex multiply-adds each, 8 flops), the update of the eight
    amplitudes (each a complex product with v_b or a scaled copy: 14 flops),
    and sin/versine with the two quotients (20 flops)."""
    lines = 8
    fft = 5 * n_r * int(np.log2(n_r))
    per_line = 4 * fft + 2 * 6 * n_r + 2 * 6 * n_r
    coupling = n_r * (2 * 3 * 8 + 8 * 14 + 20)
    return lines * per_line + coupling


def jm_bytes_per_step(n_r):
    """Algorithmic HBM bytes of one (j, m) molecule-step: the eight lines read
    and written once (complex64), the three field components, the dipole
    vector and the absorbed accumulator (read + write)."""
    return 2 * 8 * n_r * 8 + 3 * 8 + 3 * 8 + 16


def jmg_flops_per_step(n_r, j_max):
    """Algorithmic vector flops of one molecule-step in the (j, m) basis with
    2 <= j_max <= 5 ((j_max+1)^2 lines per state): four N_r-point complex
    FFTs per line, the kinetic and the two potential phase multiplies (6
    flops per point each), and at every (state, r) the rotation to the field
    frame and back (per block j >= 1: 2j+1 phase products, 6 flops, and the
    (2j+1)^2 real-by-complex products of d^j, 4 flops each); at every r the
    per-m' transforms of cos(theta) for both states, there and back (4 n^2
    real-by-complex products, n = j_max + 1 - |m'|) and the 2x2 rotation of
    each eigenvector's pair (12 flops plus 2 for the angle); and the norm and
    dipole-vector readouts (3 and about 50 flops per line and point)."""
    nb = (j_max + 1) ** 2
    lines = 2 * nb
    fft = 5 * n_r * int(np.log2(n_r))
    per_line = 4 * fft + 2 * 6 * n_r + 2 * 6 * n_r
    rot = 2 * 2 * n_r * (6 * (nb - 1) + 4 * sum((2 * j + 1) ** 2 for j in range(1, j_max + 1)))
    blocks = [j_max + 1 - abs(mp) for mp in range(-j_max, j_max + 1) if abs(mp) < j_max]
    couple = n_r * sum(16 * n * n + 14 * n for n in blocks)
    readout = 2 * nb * n_r * 3 + 50 * nb * n_r
    return lines * per_line + rot + couple + readout


def jmg_bytes_per_step(n_r, j_max):
    """Algorithmic HBM bytes of one (j, m) molecule-step: the 2 (j_max+1)^2
    lines read and written once (complex64), the three field components, the
    dipole vector and the absorbed accumulator (read + write)."""
    return 2 * 2 * (j_max + 1) ** 2 * n_r * 8 + 3 * 8 + 3 * 8 + 16


def jm_config(cfg, n_mol=691_200, n_r=256, j_max=1):
    return cfg.replace(n_mol=n_mol, j_max=j_max, basis="jm", n_r=n_r)


def mol_mfma_flops_per_step(cfg):
    """Algorithmic flops of the J->angle and angle->J contractions (a real
    n_j x n_j matrix applied to the complex wavepacket of both states)."""
    return 2 * 2 * 4 * cfg.n_j * cfg.n_j * cfg.n_r


MOL_KERNEL_SOURCES = ["common.h", "fft_reg.h", "mol.h", "mol_impl.h", "mol_mixed.hip"]


def sources_sha256():
    """Hash of the sources that define the mixed molecular kernel, to tie
    stored counter figures to the code they were taken from."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2209_04487_amd", "csrc")
    for name in MOL_KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per launch of the mixed molecular kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a copy of
    known size), or None when the kernel sources changed since."""
    try:
        with open(COUNTER_PROFILE) as f:
            text = f.read()
    except OSError:
        return None, None
    m_sha = re.search(r"sources_sha256:\s*([0-9a-f]{64})", text)
    m_t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_t):
        return None, None
    if m_sha.group(1) != sources_sha256():
        return None, "kernel sources changed since the counters were taken"
    return float(m_t.group(1)), os.path.relpath(COUNTER_PROFILE, ROOT)


def default_first_step(cfg):
    """First step of the measured window: 600 steps before the pulse peak
    leaves the source plane (the peak reaches the molecule slab about 90
    steps later), so the window covers the strong-field interaction."""
    return max(0, int(round(cfg.t0 / cfg.dt)) - 600)


def stencil_bytes_per_cell(prec):
    """Bytes per cell-update of the two stencil kernels as launched: H update
    reads E (3) and H (3), writes H (3); E update reads H (3), E (3),
    material ids (3 B), writes E (3)."""
    w = 8 if prec == "fp64" else 4
    return 18 * w + 3


def stencil_min_bytes_per_cell(prec):
    """The least a whole field step must move per cell: E and H each read
    once and written once (12 words) and the material ids (3 B), as a single
    fused H + E sweep would; the two-kernel split moves 18 words."""
    w = 8 if prec == "fp64" else 4
    return 12 * w + 3


def material_fractions(cfg):
    """(metal share of the E-component locations, averaged over the three
    components; share of the cells in the CPML slabs)."""
    from workloads.configs import MAT_METAL
    from workloads.geometry import material_map
    mat = material_map(cfg)
    return float((mat == MAT_METAL).mean()), 2.0 * cfg.npml / cfg.nz


def stencil_alg_bytes_per_cell(cfg, prec):
    """Algorithmic bytes per cell-update of a whole field step (the count the
    roofline is taken against): E and H each read and written once (12
    words), the Drude current read and written at the metal edges (2 words
    per metal E-component location, i.e. 6 words times the metal share), the
    four CPML auxiliaries read and written in the CPML slabs (8 words times
    their share of the cells), and the material ids (3 B)."""
    w = 8 if prec == "fp64" else 4
    f_metal, f_pml = material_fractions(cfg)
    return w * (12.0 + 6.0 * f_metal + 8.0 * f_pml) + 3.0


def run_coupled(cfg, prec, steps, warmup, n0, mol_every=1, time_mol=False):
    """Time `steps` coupled steps (after `warmup` untimed ones) with HIP
    events on the stream the steps are launched on.  With time_mol, the
    library also records HIP events around each molecular-step launch inside
    the timed window (msqd_mol_timing_begin/end), giving the kernel's own
    average duration in that same window."""
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.pulses import source_values
    sysm = msqd.Coupled(cfg, prec=prec, mol_every=mol_every)
    src = source_values(cfg, n0, warmup + steps)
    stream = torch.cuda.current_stream()
    if warmup:
        msqd.coupled_step(sysm.desc, sysm.state, src[:warmup], n0)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    if time_mol:
        msqd.mol_timing_begin(steps)
    t_start.record(stream)
    msqd.coupled_step(sysm.desc, sysm.state, src[warmup:], n0 + warmup)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    out = {"ms": ms, "n_mol": sysm.mol.desc.n_mol}
    if time_mol:
        mol_total, n_launch = msqd.mol_timing_end()
        out["mol_kernel_ms"] = mol_total / max(n_launch, 1)
        out["mol_launches"] = n_launch
    msqd.check_status(sysm.mol.ws)
    del sysm
    torch.cuda.empty_cache()
    return out


def run_accuracy(cfg, prec, steps, n0):
    """Untimed run of `steps` coupled steps from a fresh state, recording the
    ensemble dipole after every step; returns the trace, the transmitted
    flux spectrum and the mean dissociated population at the end."""
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.pulses import source_values
    sysm = msqd.Coupled(cfg, prec=prec)
    src = source_values(cfg, n0, steps)
    # one row of ensemble sums (dipole, norm, yield; dipole_readout) per step
    sums = torch.zeros((steps, sysm.mol.n_sums), dtype=torch.float64, device="cuda")
    for s in range(steps):
        msqd.coupled_step(sysm.desc, sysm.state, src[s:s + 1], n0 + s)
        sysm.ensemble_sums(sums[s])
    flux = sysm.fields.flux().cpu().numpy()
    msqd.check_status(sysm.mol.ws)
    sums = sums.cpu().numpy()
    out = {"D": sums[:, 0], "flux": flux, "yield": sums[-1, -1] / sysm.mol.desc.n_mol}
    del sysm
    torch.cuda.empty_cache()
    return out


def dissociating_config(cfg):
    """A variant of a workload in which the dissociation probability is a
    real signal: lighter nuclei (500 m_e), a carrier at the vertical gap
    (0.45 Eh), a short strong pulse (FWHM 2 fs, peak 5e-3 au, centred at
    3 fs) and r_diss = 4 a0, so that the excited packet crosses r_diss within
    the window.  Grid, geometry, molecules and radial/rotational basis stay
    those of the workload."""
    return cfg.replace(mass=500.0, omega_h=0.45, e0_au=5e-3, fwhm_fs=2.0, t0_steps=None, t0_fs=3.0,
                       r_diss=4.0)


def dissociating_steps(cfg):
    """Steps of the dissociating window: the pulse peak (at the slab about
    900 steps in) and 1,100 steps of dissociation after it."""
    return 2000


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_bloch(cfg, steps, warmup, n0, n_emitters):
    """Coupled step with frozen two-level emitters in place of the
    wavepackets (the paper's Bloch/RK4 comparison), timed like run_coupled;
    plus the emitter kernel alone (bloch_step on a field array)."""
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.pulses import source_values
    c = cfg.replace(n_mol=n_emitters)
    sysm = msqd.CoupledBloch(c, prec="fp32")
    src = source_values(c, n0, warmup + steps)
    sysm.n = n0
    sysm.step(src[:warmup])
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(torch.cuda.current_stream())
    sysm.step(src[warmup:])
    b.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    em = sysm.em
    E = torch.full((n_emitters,), 1e-3, dtype=torch.float64, device="cuda")
    em.step(E)
    torch.cuda.synchronize()
    a.record(torch.cuda.current_stream())
    for _ in range(20):
        em.step(E)
    b.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    kms = a.elapsed_time(b) / 20
    kbytes = n_emitters * (2 * 12 + 8 + 8)     # state in and out, field in, dipole out
    out = {"n_emitters": n_emitters, "ms_per_step": ms / steps,
           "emitter_steps_per_s": n_emitters * steps / (ms / 1e3),
           "kernel_ms": kms, "kernel_GBs": kbytes / (kms / 1e3) / 1e9,
           "kernel_frac_hbm": kbytes / (kms / 1e3) / 1e9 / HBM_PEAK_GBS}
    del sysm
    torch.cuda.empty_cache()
    return out


def run_jm(cfg, steps, warmup, n0, n_mol=691_200, n_r=256, j_max=1):
    """The paper's own molecular model: all (j, m) with j <= j_max and all
    three field components, 691,200 molecules in the SRR slab (the paper's
    count), precision form, one molecular step per field step.  j_max = 1 is
    the truncation of the paper's ensemble results (closed-form coupling);
    j_max = 5 the largest basis of its scaling test (general coupling)."""
    c = jm_config(cfg, n_mol, n_r, j_max)
    out = run_coupled(c, "fp32", steps, warmup, n0)
    rate = out["n_mol"] * steps / (out["ms"] / 1e3)
    kms = time_mol_kernel(c, "fp32", 10 if j_max == 1 else 5)
    fl = jm_flops_per_step(n_r) if j_max == 1 else jmg_flops_per_step(n_r, j_max)
    by = jm_bytes_per_step(n_r) if j_max == 1 else jmg_bytes_per_step(n_r, j_max)
    kt = fl * n_mol / (kms / 1e3) / 1e12
    kb = by * n_mol / (kms / 1e3) / 1e9
    name = f"mol_jm_kernel<float,{n_r},single-step>" if j_max == 1 else \
        f"mol_jmg_kernel<float,{n_r},{j_max},single-step>"
    return {"workload": f"SRR array, {n_mol} molecules, (j, m) basis j <= {j_max}, N_r={n_r}, FP32",
            "ms_per_step": out["ms"] / steps, "molecule_steps_per_s": rate,
            "flops_per_molecule_step": fl, "bytes_per_molecule_step": by,
            "coupled_step_TFLOPs": rate * fl / 1e12,
            "coupled_step_frac_of_vector_peak": rate * fl / 1e12 / VALU_F32_PEAK_TFLOPS,
            "kernel": name, "kernel_ms": kms,
            "kernel_TFLOPs": kt, "kernel_frac_of_vector_peak": kt / VALU_F32_PEAK_TFLOPS,
            "kernel_GBs": kb, "kernel_frac_of_hbm": kb / HBM_PEAK_GBS}


def run_scale(steps):
    """The scale workload (256 x 256 x 160 nanohole film, 700,000 molecules,
    precision form): one run, and three incident carriers (0.08, 0.09,
    0.10 Eh) advanced together as a batch on separate streams."""
    import torch

    from paper_2209_04487_amd import msqd
    from workloads import get_config
    from workloads.pulses import source_values
    cfg = get_config("cfg4")
    n0 = default_first_step(cfg)
    out = {"workload": f"nanohole film {cfg.nx}x{cfg.ny}x{cfg.nz}, {cfg.n_mol} molecules, "
                       f"N_r={cfg.n_r}, J<={cfg.j_max}, precision form"}
    one = run_coupled(cfg, "mixed", steps, 2, n0)
    out["ms_per_step"] = one["ms"] / steps
    out["molecule_steps_per_s"] = one["n_mol"] * steps / (one["ms"] / 1e3)
    cfgs = [cfg.replace(omega_h=w) for w in (0.08, 0.09, 0.10)]
    batch = msqd.CarrierBatch(cfgs, prec="mixed")
    srcs = [source_values(c, n0, steps + 2) for c in cfgs]
    for sysm in batch.systems:
        sysm.n = n0
    batch.step([s_[:2] for s_ in srcs])
    torch.cuda.synchronize()
    t = time.time()
    batch.step([s_[2:] for s_ in srcs])
    torch.cuda.synchronize()
    dt = time.time() - t
    out["carriers"] = {"n": 3, "ms_per_step_all": dt * 1e3 / steps,
                       "molecule_steps_per_s": 3 * cfg.n_mol * steps / dt}
    del batch
    torch.cuda.empty_cache()
    return out


def run_adjoint(steps, fp64_check=True):
    """Gradient of the dissociated population of the differentiation
    workload (one SRR cell, 20,000 molecules, N_r = 128, J <= 6, FP32) over a
    window of `steps` steps with one checkpoint per 200 steps: forward run,
    segment recompute and reverse steps, timed as one call.  With fp64_check
    the same gradient is also taken in the FP64 form and the FP32 yield and
    gradient are reported against it: at the workload's own parameters the
    pulse barely excites the molecules, and the comparison says whether FP32
    resolves the yield and its gradient there."""
    import torch

    from paper_2209_04487_amd.grad import yield_and_gradient
    from workloads import get_config
    from workloads.pulses import knot_values
    cfg = get_config("cfg3", n_steps=steps)
    kn = knot_values(cfg)
    yield_and_gradient(cfg.replace(n_steps=10, ckpt_every=10), kn, cfg.omega, prec="fp32")   # warm-up
    torch.cuda.synchronize()
    torch.cuda.empty_cache()      # blocks cached by earlier runs would split the 57 GB history
    t = time.time()
    Y, dk, dw = yield_and_gradient(cfg, kn, cfg.omega, prec="fp32")
    torch.cuda.synchronize()
    dt = time.time() - t
    torch.cuda.empty_cache()
    out = {"workload": f"SRR cell {cfg.nx}x{cfg.ny}x{cfg.nz}, {cfg.n_mol} molecules, N_r={cfg.n_r}, "
                       f"J<={cfg.j_max}, FP32, checkpoint every {cfg.ckpt_every}",
           "steps": steps, "s_total": dt, "ms_per_forward_plus_reverse_step": dt * 1e3 / steps,
           "yield": Y, "grad_norm_knots": float(np.linalg.norm(dk)), "dY_domega": dw}
    if fp64_check:
        t = time.time()
        Y64, dk64, dw64 = yield_and_gradient(cfg, kn, cfg.omega, prec="fp64")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        rel = {"yield": abs(Y - Y64) / abs(Y64),
               "grad_knots": float(np.abs(dk - dk64).max() / np.abs(dk64).max()),
               "dY_domega": abs(dw - dw64) / abs(dw64)}
        out["fp64"] = {"s_total": time.time() - t, "yield": Y64,
                       "grad_norm_knots": float(np.linalg.norm(dk64)), "dY_domega": dw64}
        out["fp32_vs_fp64_rel"] = rel
        out["fp32_resolves_yield"] = bool(rel["yield"] <= 1e-3)
        out["fp32_resolves_gradient"] = bool(max(rel["grad_knots"], rel["dY_domega"]) <= 1e-3)
        if not out["fp32_resolves_yield"]:
            out["note"] = ("the yield itself (FP64 value above) lies below what FP32 resolves at these parameters "
                           "(round-off of the ground-state tail beyond r_diss); the FP32 yield is throughput only")
    return out


def run_multirate(cfg, K, n0, M=40):
    """The precision form with the molecules stepped every M field steps
    (the paper's M = 40), over about K field steps from the M-aligned step
    at or before n0, after M untimed ones."""
    k_mr = max(M, (K // M) * M)
    log(f"multi-rate coupled run: molecules every {M} field steps, {k_mr} steps")
    mr = run_coupled(cfg, "mixed", k_mr, M, n0 - (n0 % M), mol_every=M)
    return {"mol_every": M, "field_steps": k_mr, "ms_per_field_step": mr["ms"] / k_mr,
            "field_steps_per_s": k_mr / (mr["ms"] / 1e3),
            "molecule_steps_per_s": mr["n_mol"] * (k_mr // M) / (mr["ms"] / 1e3)}


def calibration_copy(nbytes=1 << 30, reps=3):
    """Device-to-device copies of a known size, for scaling the HBM byte
    counters of a counter run (FETCH_SIZE / WRITE_SIZE) to bytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def time_mol_kernel(cfg, prec, launches):
    """Average duration of the fused molecular-step kernel, timed with HIP
    events on the stream it is launched on (the same kernel as in the
    coupled step, fed from a field array instead of the grid)."""
    import torch

    from paper_2209_04487_amd import msqd
    mols = msqd.Molecules.from_config(cfg, prec=prec)
    shape = (mols.desc.n_mol, 3) if cfg.basis == "jm" else (mols.desc.n_mol,)
    E = torch.full(shape, 1e-4, dtype=torch.float64, device="cuda")
    for _ in range(3):
        mols.step(E)
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(launches):
        mols.step(E)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    del mols
    torch.cuda.empty_cache()
    return ms


def time_stencil(cfg, prec, launches):
    """Average time of one field step (the H and the E update kernels) on a
    workload's grid, as the coupled step runs it: one coupled_step call of
    `launches` steps with no molecules and no monitor, timed with HIP events
    on its stream."""
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.geometry import material_map
    c = cfg.replace(n_freq=0)
    sysm = msqd.Coupled(c, prec=prec, cells=np.zeros(0, np.int32), mat=material_map(c))
    src = np.full(launches, 1.0)
    sysm.step(src[:4])
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    sysm.step(src)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    del sysm
    torch.cuda.empty_cache()
    return ms


def stencil_entry(cfg, prec, launches):
    """The field step on a workload's grid: time per step, cell updates per
    second, and the HBM fraction against the algorithmic bytes of a whole
    field step (stencil_alg_bytes_per_cell), with the bytes of the two
    kernels as launched and the bare 12-word count beside it."""
    ms = time_stencil(cfg, prec, launches)
    n_c = cfg.nx * cfg.ny * cfg.nz
    rate = n_c / (ms / 1e3)
    alg = stencil_alg_bytes_per_cell(cfg, prec)
    f_metal, f_pml = material_fractions(cfg)
    return {"grid": f"{cfg.nx}x{cfg.ny}x{cfg.nz}", "prec": prec, "kernels": "yee_h_kernel + yee_e_kernel",
            "ms_per_step": ms, "cell_updates_per_s": rate,
            "achieved_GBs": alg * rate / 1e9, "frac": alg * rate / 1e9 / HBM_PEAK_GBS,
            "bytes_per_cell": alg, "bytes_counted": ("12 words (E, H read and written once) + 6 words x metal "
                                                     f"share {f_metal:.4f} + 8 words x CPML share {f_pml:.3f} "
                                                     "+ 3 B material ids"),
            "two_kernel": {"bytes_per_cell": stencil_bytes_per_cell(prec),
                           "frac": stencil_bytes_per_cell(prec) * rate / 1e9 / HBM_PEAK_GBS},
            "fused_12_words": {"bytes_per_cell": stencil_min_bytes_per_cell(prec),
                               "frac": stencil_min_bytes_per_cell(prec) * rate / 1e9 / HBM_PEAK_GBS}}


def cpu_baseline(cfg, budget_s=20.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload (about budget_s seconds): the full-grid field update for a few
    steps and a block of 2,048 molecules for up to 30 steps; the coupled-step
    rate for all molecules is n_mol / (t_fields + n_mol * t_molecule).  The
    oracle's radial FFTs run on scipy.fft with all host threads.  Also the
    whole tiny parity run (24^3 grid, 64 molecules, 500 coupled steps) as the
    oracle computes it."""
    from oracle.coupled import CoupledOracle
    from oracle.fdtd import yee_from_config
    from oracle.molecule import model_from_config
    from workloads import get_config
    from workloads.geometry import eps_table, material_map
    from workloads.molecule_inputs import morse_v0, potentials
    from workloads.pulses import source_values
    t0 = time.time()
    yee = yee_from_config(cfg, material_map(cfg), eps_table(cfg))
    n_f = 0
    t = time.time()
    while n_f < 10 and (n_f < 2 or time.time() - t < 0.2 * budget_s):
        yee.update_H()
        yee.update_E(1.0, cfg.src_k)
        n_f += 1
    t_field = (time.time() - t) / n_f
    ug, ue, mu = potentials(cfg)
    m = model_from_config(cfg, ug, ue, mu)
    n_blk = 2048
    psi = m.initial_state(n_blk, morse_v0(cfg))
    ab = np.zeros(n_blk)
    E = np.full(n_blk, 1e-4)
    n_m = 0
    t = time.time()
    while True:
        psi, ab = m.step(psi, E, ab)
        n_m += 1
        if time.time() - t > 0.6 * budget_s or n_m >= 30:
            break
    t_mol = (time.time() - t) / (n_m * n_blk)
    rate = cfg.n_mol / (t_field + cfg.n_mol * t_mol)
    c0 = get_config("cfg0")
    t = time.time()
    CoupledOracle(c0).run(source_values(c0, 0, c0.n_steps))
    t_tiny = time.time() - t
    blas = 1
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ncpu = os.cpu_count() or 1
    return {"value": rate, "unit": "molecule-steps/s", "cores": max(ncpu, blas), "kind": "oracle",
            "cpu_count": ncpu, "cpu_model": model,
            "sample": (f"FP64 NumPy/SciPy oracle: full {cfg.nx}x{cfg.ny}x{cfg.nz} field update x{n_f} "
                       f"({t_field:.3f} s/step) and {n_blk} molecules x {n_m} steps "
                       f"({t_mol * 1e3:.3f} ms/molecule-step), combined for {cfg.n_mol} molecules; "
                       f"radial FFTs on scipy.fft with {ncpu} workers, BLAS {blas} threads, elementwise NumPy "
                       f"on one thread; {time.time() - t0:.1f} s total"),
            "tiny_parity_run": {"workload": "24^3 vacuum grid, 64 molecules, N_r=128, J<=4, 500 coupled steps",
                                "s_total": t_tiny, "molecule_steps_per_s": 64 * 500 / t_tiny}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n0", type=int, default=None,
                    help="first step of the run (default: 600 steps before the pulse peak)")
    ap.add_argument("--acc-steps", type=int, default=1000,
                    help="length of the accuracy comparison against the FP64 form (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 timing and comparison")
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the 700,000-molecule and adjoint measurements")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the differentiation workload (4,000 forward + reverse steps) and its "
                         "forward-only timing, for a kernel trace of the adjoint")
    ap.add_argument("--adjoint-steps", type=int, default=4000,
                    help="steps of the differentiation workload's gradient (4,000: the whole run; fewer for "
                         "counter runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed coupled window of the precision form (the run a kernel trace of the "
                         "headline is taken from)")
    ap.add_argument("--multirate-only", action="store_true",
                    help="only the multi-rate window (molecules every 40 field steps), for a kernel trace")
    ap.add_argument("--kernel", choices=["mixed", "fp32", "fp64", "stencil", "jm", "jm5"], default=None,
                    help="only time the molecular-step kernel of this form, or the field stencil (for counter runs), "
                         "followed by a 1 GiB calibration copy")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(see the sharding design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from workloads import get_config
    cfg = get_config("cfg2")
    cfg64 = get_config("cfg1")
    K, W = args.steps, args.warmup
    n0 = default_first_step(cfg) if args.n0 is None else args.n0
    if args.adjoint_only:
        adj = run_adjoint(args.adjoint_steps, fp64_check=not args.no_fp64)
        cfg3 = get_config("cfg3")
        fwd = run_coupled(cfg3, "fp32", 200, 20, default_first_step(cfg3))
        adj["forward_ms_per_step"] = fwd["ms"] / 200
        print(json.dumps(adj))
        return
    if args.multirate_only:
        print(json.dumps(run_multirate(cfg, K, n0)), flush=True)
        return
    if args.kernel == "stencil":
        ms = time_stencil(cfg, "mixed", K)
        cells = cfg.nx * cfg.ny * cfg.nz
        b = stencil_alg_bytes_per_cell(cfg, "mixed") * cells
        calibration_copy()
        print(json.dumps({"kernel": "stencil (H and E updates)", "launches": K, "ms": ms, "cells": cells,
                          "bytes_per_cell": b / cells, "GBs": b / (ms / 1e3) / 1e9,
                          "frac": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, "calibration_copy_bytes": 1 << 30}))
        return
    if args.kernel == "jm":
        c = jm_config(cfg)
        ms = time_mol_kernel(c, "fp32", K)
        calibration_copy()
        print(json.dumps({"kernel": "jm", "launches": K, "ms": ms, "n_mol": c.n_mol,
                          "GBs": jm_bytes_per_step(c.n_r) * c.n_mol / (ms / 1e3) / 1e9,
                          "TFLOPs": jm_flops_per_step(c.n_r) * c.n_mol / (ms / 1e3) / 1e12,
                          "calibration_copy_bytes": 1 << 30}))
        return
    if args.kernel == "jm5":
        c = jm_config(cfg, j_max=5)
        ms = time_mol_kernel(c, "fp32", K)
        calibration_copy()
        print(json.dumps({"kernel": "jm5", "launches": K, "ms": ms, "n_mol": c.n_mol,
                          "GBs": jmg_bytes_per_step(c.n_r, 5) * c.n_mol / (ms / 1e3) / 1e9,
                          "TFLOPs": jmg_flops_per_step(c.n_r, 5) * c.n_mol / (ms / 1e3) / 1e12,
                          "calibration_copy_bytes": 1 << 30}))
        return
    if args.kernel:
        c = cfg if args.kernel != "fp64" else cfg64
        ms = time_mol_kernel(c, args.kernel, K)
        b = mol_bytes_per_step(c, args.kernel) * c.n_mol
        calibration_copy()
        print(json.dumps({"kernel": args.kernel, "launches": K, "ms": ms,
                          "GBs": b / (ms / 1e3) / 1e9, "frac": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                          "TFLOPs": mol_flops_per_step(c) * c.n_mol / (ms / 1e3) / 1e12,
                          "calibration_copy_bytes": 1 << 30, "sources_sha256": sources_sha256()}))
        return

    log(f"mixed coupled run: {cfg.n_mol} molecules, {W}+{K} steps from step {n0}")
    mixed = run_coupled(cfg, "mixed", K, W, n0, time_mol=True)
    value = mixed["n_mol"] * K / (mixed["ms"] / 1e3)
    mol_ms = mixed["mol_kernel_ms"]
    unit_bytes = mol_bytes_per_step(cfg, "mixed")
    unit_flops = mol_flops_per_step(cfg)
    achieved_gbs = unit_bytes * cfg.n_mol / (mol_ms / 1e3) / 1e9
    achieved_tf = unit_flops * cfg.n_mol / (mol_ms / 1e3) / 1e12
    if args.headline_only:
        print(json.dumps({"value": value, "unit": "molecule-steps/s", "steps": K, "warmup": W,
                          "ms_per_step": mixed["ms"] / K, "mol_kernel_ms": mol_ms,
                          "mol_launches": mixed["mol_launches"], "first_step": n0,
                          "mol_kernel_TFLOPs": achieved_tf, "mol_kernel_GBs": achieved_gbs}), flush=True)
        return
    fp64 = None
    if not args.no_fp64:
        log("fp64 coupled run")
        fp64 = run_coupled(cfg64, "fp64", K, W, n0, time_mol=True)
    acc = None
    if args.acc_steps > 0 and not args.no_fp64:
        log(f"accuracy: {args.acc_steps} steps of both forms from step {n0}")
        am = run_accuracy(cfg, "mixed", args.acc_steps, n0)
        a64 = run_accuracy(cfg64, "fp64", args.acc_steps, n0)
        acc = {"steps": f"{n0}..{n0 + args.acc_steps}",
               "dipole_trace_rel_l2": rel_l2(am["D"], a64["D"]),
               "flux_spectrum_rel_l2": rel_l2(am["flux"], a64["flux"]),
               "yield_abs_err": abs(am["yield"] - a64["yield"]),
               "yield_fp64": a64["yield"], "yield_mixed": am["yield"],
               "dipole_peak_fp64": float(np.abs(a64["D"]).max())}
        # the dissociation probability is below what FP32 resolves in that
        # window (the ground-state tail beyond r_diss); a dissociating variant
        # of the same geometry and pulse shape makes it a real signal
        dc = dissociating_config(cfg)
        n_d = dissociating_steps(dc)
        log(f"accuracy, dissociating variant: {n_d} steps of both forms")
        dm = run_accuracy(dc, "mixed", n_d, 0)
        d64 = run_accuracy(dc.replace(precision="fp64"), "fp64", n_d, 0)
        acc["dissociating_variant"] = {
            "workload": (f"same grid, molecules and pulse shape; reduced mass {dc.mass:g} m_e, carrier "
                         f"{dc.omega_h:g} Eh at the vertical gap, peak {dc.e0_au:g} au, r_diss {dc.r_diss:g} a0, "
                         f"steps 0..{n_d}"),
            "yield_fp64": d64["yield"], "yield_mixed": dm["yield"],
            "yield_rel_err": abs(dm["yield"] - d64["yield"]) / abs(d64["yield"]),
            "dipole_trace_rel_l2": rel_l2(dm["D"], d64["D"]),
            "flux_spectrum_rel_l2": rel_l2(dm["flux"], d64["flux"])}

    multirate = run_multirate(cfg, K, n0)

    log("(j, m)-basis coupled run: 691,200 molecules, j <= 1")
    jm = run_jm(cfg, 20, 2, n0)
    log("(j, m)-basis coupled run: 691,200 molecules, j <= 1, N_r = 512 (the paper's radial grid size)")
    jm["n_r_512"] = run_jm(cfg, 10, 1, n0, n_r=512)
    log("(j, m)-basis coupled run: 691,200 molecules, j <= 5")
    try:
        jm["j_max_5"] = run_jm(cfg, 5, 1, n0, j_max=5)
    except torch.cuda.OutOfMemoryError as e:       # 102 GB of wavepackets: report, do not lose the line
        torch.cuda.empty_cache()
        jm["j_max_5"] = {"error": f"out of device memory: {e}".splitlines()[0]}
    log("Bloch-emitter coupled run: 691,200 emitters")
    bloch = run_bloch(cfg, K, W, n0, 691_200)

    # coupled-step rates of the other two workloads: the tiny parity case
    # (64 molecules, FP64; launch-latency bound) and the differentiation
    # cell's forward step (20,000 molecules, FP32)
    other = {}
    for name, pr in (("cfg0", "fp64"), ("cfg3", "fp32")):
        c = get_config(name)
        o = run_coupled(c, pr, max(K, 50), W, default_first_step(c))
        other[name] = {"workload": f"{c.nx}x{c.ny}x{c.nz} cells, {c.n_mol} molecules, N_r={c.n_r}, "
                                   f"J<={c.j_max}, {pr}",
                       "ms_per_step": o["ms"] / max(K, 50),
                       "molecule_steps_per_s": o["n_mol"] * max(K, 50) / (o["ms"] / 1e3),
                       "cell_updates_per_s": c.nx * c.ny * c.nz * max(K, 50) / (o["ms"] / 1e3)}

    scale = None
    adjoint = None
    if not args.no_scale:
        log("scale workload: 700,000 molecules, one run and a 3-carrier batch")
        scale = run_scale(10)
        log("adjoint: differentiation workload, 4,000 steps, FP32 and FP64")
        adjoint = run_adjoint(4000, fp64_check=not args.no_fp64)

    log("stencil timing")
    launches = max(10, min(K, 100))
    traffic, traffic_src = counter_traffic()
    cells = cfg.nx * cfg.ny * cfg.nz
    stencil = stencil_entry(cfg, "mixed", launches)
    # cell-updates/s of the other grids: the differentiation cell (FP32), the
    # nanohole film (precision form) and the SRR grid in FP64
    stencil["other_grids"] = {name: stencil_entry(get_config(name), pr, launches)
                              for name, pr in (("cfg3", "fp32"), ("cfg4", "mixed"), ("cfg1", "fp64"))}

    cpu = None
    if not args.no_cpu:
        log("cpu oracle baseline")
        cpu = cpu_baseline(cfg64)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "molecule-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": mixed["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16x3 (f64 reductions)",
        "data": "synthetic",
        "config": {
            "workload": (f"SRR array {cfg.nx}x{cfg.ny}x{cfg.nz} cells dx=2nm, {cfg.n_mol} molecules, "
                         f"N_r={cfg.n_r}, J<={cfg.j_max}, precision form"),
            "n_mol": cfg.n_mol, "n_r": cfg.n_r, "j_max": cfg.j_max, "cells": cells,
            "first_step": n0,
        },
        "roofline": {
            "bound": "alu", "achieved": achieved_tf, "peak": VALU_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved_tf / VALU_F32_PEAK_TFLOPS,
            "traffic": None if traffic is None else traffic,
            "traffic_source": traffic_src,
            "kernel": "mol_step_kernel<float,256,bf16x3,single-step>", "kernel_ms": mol_ms,
            "kernel_ms_source": (f"HIP events around each of the {mixed['mol_launches']} molecular-step launches "
                                 f"inside the timed window, on the coupled step's stream"),
            "flops_per_molecule_step": unit_flops,
            "mfma_flops_per_molecule_step": mol_mfma_flops_per_step(cfg),
            "mfma": {"achieved": mol_mfma_flops_per_step(cfg) * cfg.n_mol / (mol_ms / 1e3) / 1e12,
                     "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": mol_mfma_flops_per_step(cfg) * cfg.n_mol / (mol_ms / 1e3) / 1e12
                     / BF16_MFMA_PEAK_TFLOPS,
                     "counted": "the J<->angle contractions at N_J; not the three BF16 products per "
                                "contraction nor the padding of N_J to 16"},
            "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved_gbs / HBM_PEAK_GBS, "bytes_per_molecule_step": unit_bytes,
                    "algorithmic_bytes_per_launch": unit_bytes * cfg.n_mol},
        },
        "stencil": stencil,
        "fp64": None if fp64 is None else {
            "value": fp64["n_mol"] * K / (fp64["ms"] / 1e3), "ms_per_step": fp64["ms"] / K,
            "mol_kernel_ms": fp64["mol_kernel_ms"]},
        "speedup_vs_fp64": None if fp64 is None else fp64["ms"] / mixed["ms"],
        "accuracy_vs_fp64": acc,
        "multirate": multirate,
        "jm_basis": jm,
        "bloch_emitters": bloch,
        "other_workloads": other,
        "scale": scale,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
