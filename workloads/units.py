"""CODATA 2018 constants used to build inputs (SI and Hartree atomic units)."""

C0 = 299792458.0                 # m/s
EPS0 = 8.8541878128e-12          # F/m
MU0 = 1.25663706212e-6           # H/m
ETA0 = 376.730313668             # ohm
E_AU = 5.14220674763e11          # V/m per atomic unit of field
T_AU = 2.4188843265857e-17       # s per atomic unit of time
EA0 = 8.4783536255e-30           # C m per atomic unit of dipole (e a0)
HARTREE_EV = 27.211386245988     # eV per hartree
HBAR_EVS = 6.582119569e-16       # eV s
FS = 1.0e-15                     # s


def ev_to_rad_s(e_ev):
    """Angular frequency (rad/s) of a photon energy given in eV."""
    return e_ev / HBAR_EVS


def hartree_to_rad_s(e_h):
    """Angular frequency (rad/s) of a photon energy given in hartree."""
    return e_h / T_AU
