"""The five synthetic workloads (tiny parity case, FP64 and mixed SRR array,
differentiation case, nanohole scale case) as frozen dataclasses.

Every number here is either stated for the workload or is one of the readings
recorded in the design notes (radial-grid convention, z layout, CPML grading,
monitor frequencies, seeds).
"""

from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

from . import units as U

# material ids, one per E-component location
MAT_VACUUM = 0
MAT_GLASS = 1
MAT_METAL = 2


@dataclass(frozen=True)
class Config:
    name: str
    # Yee grid (SI)
    nx: int
    ny: int
    nz: int
    dx: float                      # m, cubic cells
    courant: float = 0.5           # c dt / dx
    npml: int = 6
    cpml_m: float = 3.0            # polynomial grading order
    cpml_kappa_max: float = 1.0
    cpml_alpha_max: float = 0.0
    eps_lo: float = 1.0            # background permittivity of the low-z CPML
    eps_hi: float = 1.0            # background permittivity of the high-z CPML
    # materials
    eps_glass: float = 2.25
    eps_inf: float = 3.7
    drude_wp_ev: float = 9.1
    drude_gamma_ev: float = 0.018
    geometry: str = "vacuum"       # vacuum | srr | nanohole
    geom: dict = field(default_factory=dict)
    # source and monitor planes
    src_k: int = 7
    mon_k: int = 16
    n_freq: int = 32
    freq_lo_h: float = 0.05
    freq_hi_h: float = 0.15
    mon_every: int = 4
    mon_k2: int = 0                # incident-side detection plane (0 = none)
    # molecules
    n_mol: int = 64
    placement: str = "block"       # block | slab
    block_lo: int = 10
    block_n: int = 4
    slab_k0: int = 0
    slab_nk: int = 0
    seed: int = 0
    mol_weight: float = 1.0
    # molecular model (atomic units)
    n_r: int = 128
    r_min: float = 1.0
    r_max: float = 12.0
    j_max: int = 4
    basis: str = "m0"              # m0: J lines, field along the axis | jm: all (j, m), 1 <= j_max <= 5
    mass: float = 1.0e4
    morse_d: float = 0.17
    morse_a: float = 1.0
    morse_re: float = 2.0
    morse_shift: bool = False      # True: subtract D so that U_g(r_e) = -D
    ue_c0: float = 0.17
    ue_c1: float = 0.30
    ue_b: float = 1.2
    ue_r0: float = 2.0
    mu_b: float = 0.1
    mu_r0: float = 2.0
    absorb_width: float = 2.0
    r_diss: float = 8.0
    # incident pulse
    pulse: str = "gauss"           # gauss | knots | cw
    cw_ramp_fs: float = 5.0        # CW drive: sin^2 turn-on time
    omega_h: float = 0.10          # carrier, hartree
    fwhm_fs: float = 10.0
    e0_au: float = 1.0e-3
    t0_steps: float | None = 250.0  # pulse centre in steps (tiny case) ...
    t0_fs: float | None = None      # ... or in fs
    n_knots: int = 64
    knot_seed: int = 4
    # run
    n_steps: int = 500
    precision: str = "fp64"        # fp64 | fp32 | mixed
    ckpt_every: int = 200

    # ---- derived quantities -------------------------------------------------
    @property
    def dt(self) -> float:
        """FDTD time step in seconds (Courant number times dx / c)."""
        return self.courant * self.dx / U.C0

    @property
    def dt_au(self) -> float:
        """The same step in atomic units of time (the molecular step)."""
        return self.dt / U.T_AU

    @property
    def n_j(self) -> int:
        return self.j_max + 1

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def t0(self) -> float:
        if self.t0_fs is not None:
            return self.t0_fs * U.FS
        return self.t0_steps * self.dt

    @property
    def omega(self) -> float:
        return U.hartree_to_rad_s(self.omega_h)

    @property
    def wp(self) -> float:
        return U.ev_to_rad_s(self.drude_wp_ev)

    @property
    def gamma(self) -> float:
        return U.ev_to_rad_s(self.drude_gamma_ev)

    def sigma_max(self, eps_bg: float) -> float:
        """Polynomial-graded CPML conductivity maximum for a background eps."""
        return 0.8 * (self.cpml_m + 1.0) / (U.ETA0 * self.dx * math.sqrt(eps_bg))

    @property
    def sigma_max_lo(self) -> float:
        return self.sigma_max(self.eps_lo)

    @property
    def sigma_max_hi(self) -> float:
        return self.sigma_max(self.eps_hi)

    @property
    def freqs(self):
        """Monitor angular frequencies (rad/s), uniform in [freq_lo, freq_hi] Eh."""
        if self.n_freq == 1:
            return [U.hartree_to_rad_s(self.freq_lo_h)]
        step = (self.freq_hi_h - self.freq_lo_h) / (self.n_freq - 1)
        return [U.hartree_to_rad_s(self.freq_lo_h + f * step) for f in range(self.n_freq)]

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


_SRR_GEOM = dict(cell=48, outer=40, arm=10, gap=10, z0=64, z1=84, glass_k=84)

CONFIGS: dict[str, Config] = {
    # tiny plain FP64 parity case
    "cfg0": Config(
        name="cfg0", nx=24, ny=24, nz=24, dx=5e-9, npml=6, geometry="vacuum",
        src_k=7, mon_k=16, n_mol=64, placement="block", block_lo=10, block_n=4,
        n_r=128, j_max=4, t0_steps=250.0, n_steps=500, precision="fp64"),
    # SRR array, plain FP64
    "cfg1": Config(
        name="cfg1", nx=192, ny=192, nz=120, dx=2e-9, npml=12, eps_hi=2.25,
        geometry="srr", geom=dict(_SRR_GEOM), src_k=16, mon_k=100,
        n_mol=100_000, placement="slab", slab_k0=54, slab_nk=10, seed=1,
        n_r=256, j_max=10, t0_steps=None, t0_fs=20.0, n_steps=20_000,
        precision="fp64"),
    # same geometry and seed, precision form
    "cfg2": Config(
        name="cfg2", nx=192, ny=192, nz=120, dx=2e-9, npml=12, eps_hi=2.25,
        geometry="srr", geom=dict(_SRR_GEOM), src_k=16, mon_k=100,
        n_mol=100_000, placement="slab", slab_k0=54, slab_nk=10, seed=1,
        n_r=256, j_max=10, t0_steps=None, t0_fs=20.0, n_steps=20_000,
        precision="mixed"),
    # differentiation case: one SRR unit cell, FP32, 64-knot envelope
    "cfg3": Config(
        name="cfg3", nx=96, ny=96, nz=80, dx=2e-9, npml=12, eps_hi=2.25,
        geometry="srr", geom=dict(cell=96, outer=40, arm=10, gap=10, z0=40, z1=60,
                                  glass_k=60),
        src_k=16, mon_k=64, n_mol=20_000, placement="slab", slab_k0=30,
        slab_nk=10, seed=3, n_r=128, j_max=6, pulse="knots", n_knots=64,
        knot_seed=4, t0_steps=None, t0_fs=0.0, n_steps=4000, precision="fp32",
        ckpt_every=200),
    # scale case: perforated film, 700k molecules, precision form
    "cfg4": Config(
        name="cfg4", nx=256, ny=256, nz=160, dx=2e-9, npml=12, eps_hi=2.25,
        geometry="nanohole", geom=dict(centres=((50, 50), (150, 50), (50, 150),
                                                (150, 150)), side=60, z0=75,
                                       z1=100, glass_k=100),
        src_k=16, mon_k=140, n_mol=700_000, placement="slab", slab_k0=60,
        slab_nk=15, seed=5, n_r=256, j_max=10, t0_steps=None, t0_fs=20.0,
        n_steps=20_000, precision="mixed"),
}


def get_config(name: str, **overrides) -> Config:
    cfg = CONFIGS[name]
    return cfg.replace(**overrides) if overrides else cfg
