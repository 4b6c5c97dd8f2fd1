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
comparison, and the relative L2 error of the ensemble dipole trace of the
precision form against the FP64 form is measured over the same steps.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
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


def stencil_bytes_per_cell(prec):
    """Algorithmic bytes per cell-update of the two stencil kernels as
    launched: H update reads E (3) and H (3), writes H (3); E update reads H
    (3), E (3), material ids (3 B), writes E (3)."""
    w = 8 if prec == "fp64" else 4
    return 18 * w + 3


def run_coupled(cfg, prec, steps, warmup, n0, record_d):
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.pulses import source_values
    sysm = msqd.Coupled(cfg, prec=prec)
    src = source_values(cfg, n0, warmup + steps)
    stream = torch.cuda.current_stream()
    # warm-up steps (part of the same run)
    if warmup:
        msqd.coupled_step(sysm.desc, sysm.state, src[:warmup], n0)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    msqd.coupled_step(sysm.desc, sysm.state, src[warmup:], n0 + warmup)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    msqd.check_status(sysm.mol.ws)
    D = None
    if record_d:
        # untimed replay of the same steps from a fresh state, recording the
        # ensemble dipole after every step
        del sysm
        torch.cuda.empty_cache()
        sysm = msqd.Coupled(cfg, prec=prec)
        D = np.zeros(warmup + steps)
        acc = torch.zeros(warmup + steps, dtype=torch.float64, device="cuda")
        for s in range(warmup + steps):
            msqd.coupled_step(sysm.desc, sysm.state, src[s:s + 1], n0 + s)
            acc[s] = sysm.mol.d.sum()
        D = acc.cpu().numpy()
    out = {"ms": ms, "D": D, "n_mol": sysm.mol.desc.n_mol}
    del sysm
    torch.cuda.empty_cache()
    return out


def time_mol_kernel(cfg, prec, launches):
    """Average duration of the fused molecular-step kernel, timed with HIP
    events on the stream it is launched on (the same kernel as in the
    coupled step, fed from a field array instead of the grid)."""
    import torch

    from paper_2209_04487_amd import msqd
    mols = msqd.Molecules.from_config(cfg, prec=prec)
    E = torch.full((mols.desc.n_mol,), 1e-4, dtype=torch.float64, device="cuda")
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
    import torch

    from paper_2209_04487_amd import msqd
    from workloads.geometry import material_map
    fl = msqd.Fields(msqd.fdtd_desc_from_config(cfg, prec, n_freq=0), material_map(cfg), [])
    for n in range(3):
        fl.step(n, 0.0)
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for n in range(launches):
        fl.step(n, 1.0)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / launches
    del fl
    torch.cuda.empty_cache()
    return ms


def cpu_baseline(cfg, budget_s=20.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: the full-grid field update for a few steps and a block of
    molecules for a few steps; the coupled-step rate for all molecules is
    n_mol / (t_fields + n_mol * t_molecule)."""
    from oracle.fdtd import yee_from_config
    from oracle.molecule import model_from_config
    from workloads.geometry import eps_table, material_map
    from workloads.molecule_inputs import morse_v0, potentials
    t0 = time.time()
    yee = yee_from_config(cfg, material_map(cfg), eps_table(cfg))
    n_f = 2
    t = time.time()
    for _ in range(n_f):
        yee.update_H()
        yee.update_E(1.0, cfg.src_k)
    t_field = (time.time() - t) / n_f
    ug, ue, mu = potentials(cfg)
    m = model_from_config(cfg, ug, ue, mu)
    n_blk = 256
    psi = m.initial_state(n_blk, morse_v0(cfg))
    ab = np.zeros(n_blk)
    E = np.full(n_blk, 1e-4)
    n_m = 0
    t = time.time()
    while True:
        psi, ab = m.step(psi, E, ab)
        n_m += 1
        if time.time() - t > min(budget_s / 2, 8.0) or n_m >= 20:
            break
    t_mol = (time.time() - t) / (n_m * n_blk)
    rate = cfg.n_mol / (t_field + cfg.n_mol * t_mol)
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        pass
    return {"value": rate, "unit": "molecule-steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle: full {cfg.nx}x{cfg.ny}x{cfg.nz} field update x{n_f} "
                       f"({t_field:.3f} s/step) and {n_blk} molecules x {n_m} steps "
                       f"({t_mol * 1e3:.3f} ms/molecule-step), combined for {cfg.n_mol} molecules; "
                       f"FFTs single-threaded, BLAS {threads} threads; {time.time() - t0:.1f} s total")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n0", type=int, default=0, help="first step of the run (pulse time origin)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--kernel", choices=["mixed", "fp32", "fp64"], default=None,
                    help="only time the molecular-step kernel of this form (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
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
    if args.kernel:
        ms = time_mol_kernel(cfg, args.kernel, K)
        b = mol_bytes_per_step(cfg, args.kernel) * cfg.n_mol
        print(json.dumps({"kernel": args.kernel, "launches": K, "ms": ms,
                          "GBs": b / (ms / 1e3) / 1e9, "frac": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}))
        return

    log(f"mixed coupled run: {cfg.n_mol} molecules, {W}+{K} steps")
    mixed = run_coupled(cfg, "mixed", K, W, args.n0, record_d=not args.no_fp64)
    value = mixed["n_mol"] * K / (mixed["ms"] / 1e3)
    fp64 = None
    err = None
    if not args.no_fp64:
        log("fp64 coupled run")
        fp64 = run_coupled(cfg64, "fp64", K, W, args.n0, record_d=True)
        D64, Dm = fp64["D"], mixed["D"]
        err = float(np.linalg.norm(Dm - D64) / max(np.linalg.norm(D64), 1e-300))

    log("kernel timing")
    launches = max(10, min(K, 100))
    mol_ms = time_mol_kernel(cfg, "mixed", launches)
    unit_bytes = mol_bytes_per_step(cfg, "mixed")
    achieved = unit_bytes * cfg.n_mol / (mol_ms / 1e3) / 1e9
    sten_ms = time_stencil(cfg, "mixed", launches)
    cells = cfg.nx * cfg.ny * cfg.nz
    sten_gbs = stencil_bytes_per_cell("mixed") * cells / (sten_ms / 1e3) / 1e9
    mol64_ms = time_mol_kernel(cfg64, "fp64", max(5, launches // 4)) if not args.no_fp64 else None

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
        "dtype": "f32+bf16 (f64 reductions)",
        "data": "synthetic",
        "config": {
            "workload": (f"SRR array {cfg.nx}x{cfg.ny}x{cfg.nz} cells dx=2nm, {cfg.n_mol} molecules, "
                         f"N_r={cfg.n_r}, J<={cfg.j_max}, precision form"),
            "n_mol": cfg.n_mol, "n_r": cfg.n_r, "j_max": cfg.j_max, "cells": cells,
            "first_step": args.n0,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "mol_step_kernel<float,256,mfma>", "kernel_ms": mol_ms,
            "bytes_per_molecule_step": unit_bytes,
        },
        "stencil": {"ms_per_step": sten_ms, "cell_updates_per_s": cells / (sten_ms / 1e3),
                    "achieved_GBs": sten_gbs, "frac": sten_gbs / HBM_PEAK_GBS},
        "fp64": None if fp64 is None else {
            "value": fp64["n_mol"] * K / (fp64["ms"] / 1e3), "ms_per_step": fp64["ms"] / K,
            "mol_kernel_ms": mol64_ms},
        "speedup_vs_fp64": None if fp64 is None else fp64["ms"] / mixed["ms"],
        "dipole_rel_err_vs_fp64": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
