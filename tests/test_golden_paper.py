"""Worked numbers printed in the paper, recomputed from the unit conversions
and model curves the build uses."""

import json
import math
import os

import numpy as np

from workloads import get_config
from workloads import units as U

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_grid_point_count():
    g = GOLDEN["fdtd_grid"]
    assert g["nx"] * g["ny"] * g["nz"] > g["at_least_points"]


def test_iteration_count_from_time_step():
    g = GOLDEN["fdtd_time"]
    cfg = get_config("cfg0", dx=g["dx_m"], courant=g["courant"])
    n = g["t_total_fs"] * U.FS / cfg.dt
    assert abs(n / g["iterations"] - 1) < g["rel_tol"]


def test_molecular_layer_and_update_interval():
    g = GOLDEN["molecular_layer"]
    layers = round(g["thickness_m"] / GOLDEN["fdtd_time"]["dx_m"])
    assert GOLDEN["fdtd_grid"]["nx"] * GOLDEN["fdtd_grid"]["ny"] * layers == g["molecules"]
    m = GOLDEN["molecular_update"]
    cfg = get_config("cfg0", dx=GOLDEN["fdtd_time"]["dx_m"], courant=0.5)
    assert abs(m["every"] * cfg.dt / (m["interval_fs"] * U.FS) - 1) < m["rel_tol"]


def test_li2_vertical_gap():
    """At R_g the shifted Morse of Eq. (6) sits at -D_g and Eq. (7) gives the
    excited surface; the difference is the ~1.5 eV SPPR-matched gap."""
    g = GOLDEN["li2_gap"]
    cfg = get_config("cfg0", n_r=512, r_min=3.0, r_max=50.0, morse_d=g["D_g"],
                     morse_a=g["alpha_g"], morse_re=g["R_g"], morse_shift=True,
                     ue_c0=0.0, ue_c1=2 * g["D_e"], ue_b=g["alpha_e"], ue_r0=g["R_e"])
    from workloads.molecule_inputs import potentials, r_grid
    r = r_grid(cfg)
    ug, ue, _ = potentials(cfg)
    k = int(np.argmin(np.abs(r - g["R_g"])))
    gap = np.interp(g["R_g"], r, ue) - np.interp(g["R_g"], r, ug)
    assert abs(ug[np.argmin(ug)] + g["D_g"]) < 1e-3
    assert abs(gap * U.HARTREE_EV - g["gap_eV"]) < g["abs_tol_eV"], gap * U.HARTREE_EV
    assert k > 0


def test_drude_frequency_conversion():
    g = GOLDEN["au_drude"]
    assert abs(U.ev_to_rad_s(g["wp_eV"]) / 1.3711e16 - 1) < 1e-3
    assert math.isclose(U.ev_to_rad_s(1.0) * U.HBAR_EVS, 1.0)
