"""Full-length certification of the plain FP64 GPU form against the oracle on
the 100,000-molecule SRR workload (192 x 192 x 120 grid, N_r = 256, J <= 10).

Two parts, each longer than a test may run:

* decoupled replay: the whole 20,000-step FP64 coupled run on the GPU records,
  for 64 seeded molecules (the last one included), the field each of them saw
  at every step and its dipole after the step; the oracle then propagates the
  same 64 molecules from the same Morse start under those fields for all
  20,000 steps, and the dipoles are compared at every step (and the final
  wavepackets and absorbed norms at the end);
* field solver alone on the same grid for 2,000 steps, with the workload's
  pulse shortened (FWHM 4 fs, centred at 6 fs) so that its peak crosses the
  split rings, the slab, the glass and the upper CPML inside the window:
  all six components on four z planes (below the source, the molecule slab,
  the rings, the glass at the detection plane) after 500, 1,000 and 2,000
  steps against the oracle's.

Usage (not collected by pytest):
  python tests/certify_full_length.py gpu OUT.npz      # on the GPU, a few minutes
  python tests/certify_full_length.py oracle OUT.npz   # on the host, the oracle side
The oracle side prints the errors; the criterion is 1e-10 relative to each
quantity's peak.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

N_STEPS = 20_000
N_SAMPLE = 64
FIELD_STEPS = 2000
FIELD_CHECKS = (500, 1000, 2000)
PLANES = (13, 59, 74, 100)
COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def _log(msg):
    print(f"[certify] {msg}", flush=True)


def sample_molecules(n_mol):
    rng = np.random.default_rng(2024)
    s = np.sort(rng.choice(n_mol - 1, N_SAMPLE - 1, replace=False))
    return np.concatenate([s, [n_mol - 1]]).astype(np.int64)


def field_config():
    from workloads import get_config
    return get_config("cfg1", fwhm_fs=4.0, t0_fs=6.0, n_freq=0)


def run_gpu(out_path):
    import torch

    from paper_2209_04487_amd import msqd
    from workloads import get_config
    from workloads.geometry import material_map
    from workloads.pulses import source_values
    cfg = get_config("cfg1")
    sysm = msqd.Coupled(cfg, prec="fp64")
    idx_np = sample_molecules(cfg.n_mol)
    idx = torch.as_tensor(idx_np, device="cuda")
    src = source_values(cfg, 0, N_STEPS)
    E_rec = torch.zeros((N_STEPS, N_SAMPLE), dtype=torch.float64, device="cuda")
    d_rec = torch.zeros((N_STEPS, N_SAMPLE), dtype=torch.float64, device="cuda")
    sums = torch.zeros((N_STEPS, sysm.mol.n_sums), dtype=torch.float64, device="cuda")
    t0 = time.time()
    for t in range(N_STEPS):
        sysm.step(src[t:t + 1])
        E_rec[t] = sysm.E_mol[idx]
        d_rec[t] = sysm.mol.d[idx]
        sysm.ensemble_sums(sums[t])
        if (t + 1) % 1000 == 0:
            torch.cuda.synchronize()
            _log(f"coupled FP64 step {t + 1}/{N_STEPS} ({time.time() - t0:.0f} s)")
    msqd.check_status(sysm.mol.ws)
    out = {"sample": idx_np, "E_mol": E_rec.cpu().numpy(), "d": d_rec.cpu().numpy(),
           "psi": sysm.mol.psi[idx].cpu().numpy(), "absorbed": sysm.mol.absorbed[idx].cpu().numpy(),
           "ensemble_sums": sums.cpu().numpy()}
    del sysm
    torch.cuda.empty_cache()

    fc = field_config()
    fl = msqd.Fields(msqd.fdtd_desc_from_config(fc, "fp64", n_freq=0), material_map(fc), [])
    fsrc = source_values(fc, 0, FIELD_STEPS)
    for n in range(FIELD_STEPS):
        fl.step(n, fsrc[n])
        if n + 1 in FIELD_CHECKS:
            for c in COMPONENTS:
                out[f"{c}_{n + 1}"] = getattr(fl, c)[list(PLANES)].cpu().numpy()
            _log(f"fields step {n + 1}")
    np.savez(out_path, **out)
    _log(f"wrote {out_path}")


def run_oracle(in_path, part):
    from oracle.fdtd import yee_from_config
    from oracle.molecule import model_from_config
    from workloads import get_config
    from workloads.geometry import eps_table, material_map
    from workloads.molecule_inputs import morse_v0, potentials
    from workloads.pulses import source_values
    rec = np.load(in_path)
    if part in ("replay", "all"):
        cfg = get_config("cfg1")
        m = model_from_config(cfg, *potentials(cfg))
        psi = m.initial_state(N_SAMPLE, morse_v0(cfg))
        ab = np.zeros(N_SAMPLE)
        E = rec["E_mol"]
        d_gpu = rec["d"]
        d_or = np.zeros_like(d_gpu)
        t0 = time.time()
        for t in range(N_STEPS):
            psi, ab = m.step(psi, E[t], ab)
            d_or[t] = m.dipole(psi)
            if (t + 1) % 2000 == 0:
                _log(f"replay step {t + 1}/{N_STEPS} ({time.time() - t0:.0f} s)")
        peak = np.abs(d_or).max()
        err_t = np.abs(d_gpu - d_or).max(axis=1) / peak
        psi_err = np.abs(rec["psi"] - psi).max() / np.abs(psi).max()
        ab_err = np.abs(rec["absorbed"] - ab).max() / max(np.abs(ab).max(), 1e-300)
        _log(f"replay: dipoles over {N_STEPS} steps, largest error {err_t.max():.3e} of the peak "
             f"(at step {int(err_t.argmax())}), peak {peak:.3e} e a0; final wavepackets {psi_err:.3e} of the peak; "
             f"absorbed {ab_err:.3e} of the largest ({np.abs(ab).max():.3e})")
        for w in range(0, N_STEPS, 2000):
            _log(f"  steps {w}..{w + 2000}: {err_t[w:w + 2000].max():.3e}")
    if part in ("fields", "all"):
        fc = field_config()
        yee = yee_from_config(fc, material_map(fc), eps_table(fc))
        fsrc = source_values(fc, 0, FIELD_STEPS)
        t0 = time.time()
        for n in range(FIELD_STEPS):
            yee.update_H()
            yee.update_E(fsrc[n], fc.src_k)
            if n + 1 in FIELD_CHECKS:
                emax = max(np.abs(e).max() for e in yee.E)
                hmax = max(np.abs(h).max() for h in yee.H)
                errs = []
                for c, nm in enumerate(COMPONENTS):
                    ref = (yee.E if c < 3 else yee.H)[c % 3][list(PLANES)]
                    scale = emax if c < 3 else hmax
                    errs.append(np.abs(rec[f"{nm}_{n + 1}"] - ref).max() / scale)
                _log(f"fields step {n + 1}: " + ", ".join(f"{nm} {e:.2e}" for nm, e in zip(COMPONENTS, errs))
                     + f" (of the E peak {emax:.3e} V/m and H peak {hmax:.3e} A/m; {time.time() - t0:.0f} s)")
            elif (n + 1) % 100 == 0:
                _log(f"fields step {n + 1}/{FIELD_STEPS} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    if len(sys.argv) < 3 or sys.argv[1] not in ("gpu", "oracle"):
        print(__doc__)
        sys.exit(2)
    if sys.argv[1] == "gpu":
        run_gpu(sys.argv[2])
    else:
        run_oracle(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "all")
