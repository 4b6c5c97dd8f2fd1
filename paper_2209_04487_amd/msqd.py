"""Python binding of libmsqd (ctypes).

Argument marshalling only: every step of the path runs in the HIP library.
torch provides device memory and the stream.  The entry points keep the C
names (qd_init, qd_step, dipole_readout, fdtd_init, fdtd_step, flux_readout,
spectra_readout, map_build, coupled_step, adjoint_step, ...); the classes
below only allocate the buffers the C calls expect and hold the descriptors.
Every number a caller reads back (dipoles, ensemble sums, <R>_e, spectra)
is computed by the library; this module does no arithmetic on them.

The library is loaded from this package directory; if it is missing the import
fails loudly (there is no fallback implementation).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsqd.so")

MSQD_OK, MSQD_EINVAL, MSQD_ESHAPE, MSQD_EPREC, MSQD_EUNSUP, MSQD_EDEVICE, MSQD_ENONFINITE = (
    0, -1, -2, -3, -4, -5, -6)
FP64, FP32, MIXED = 0, 1, 2
PREC = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
BASIS_M0, BASIS_JM = 0, 1
BASIS = {"m0": BASIS_M0, "jm": BASIS_JM}

# CODATA 2018 (for converting readouts; the library has its own copy)
E_AU = 5.14220674763e11
EA0 = 8.4783536255e-30

EXPORTS = ["msqd_last_error", "msqd_version", "qd_workspace_bytes", "qd_init", "qd_step",
           "dipole_readout", "msqd_check_status", "fdtd_workspace_bytes", "fdtd_psi_bytes",
           "fdtd_dft_bytes", "fdtd_init", "fdtd_step", "flux_readout", "map_build", "map_csr", "map_planes",
           "coupled_step", "adjoint_scratch_bytes", "adjoint_init_yield", "adjoint_step",
           "bloch_init", "bloch_step", "coupled_bloch_step", "excited_r_readout", "qd_jm_tables_size",
           "qd_jm_tables", "spectra_readout", "msqd_mol_timing_begin", "msqd_mol_timing_end", "dipole_readout_noalloc"]


class MsqdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"msqd error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmsqd.so not found at {LIB_PATH}; build it with "
                      "python -m paper_2209_04487_amd.build")
lib = C.CDLL(LIB_PATH)


class qd_desc(C.Structure):
    _fields_ = [("n_mol", C.c_int32), ("n_r", C.c_int32), ("j_max", C.c_int32),
                ("prec", C.c_int32), ("r_min", C.c_double), ("r_max", C.c_double),
                ("mass_au", C.c_double), ("dt_au", C.c_double),
                ("absorb_width_au", C.c_double), ("r_diss_au", C.c_double),
                ("basis", C.c_int32)]


class fdtd_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("npml", C.c_int32),
                ("prec", C.c_int32), ("metal_id", C.c_int32), ("dx", C.c_double),
                ("dt", C.c_double), ("eps_r", C.c_double * 4), ("drude_wp", C.c_double),
                ("drude_gamma", C.c_double), ("cpml_m", C.c_double),
                ("sigma_max_lo", C.c_double), ("sigma_max_hi", C.c_double),
                ("kappa_max", C.c_double), ("alpha_max", C.c_double), ("src_k", C.c_int32),
                ("mon_k", C.c_int32), ("n_freq", C.c_int32), ("mon_every", C.c_int32),
                ("mon_k2", C.c_int32)]


class fdtd_fields(C.Structure):
    _fields_ = [("Ex", C.c_void_p), ("Ey", C.c_void_p), ("Ez", C.c_void_p),
                ("Hx", C.c_void_p), ("Hy", C.c_void_p), ("Hz", C.c_void_p),
                ("JDx", C.c_void_p), ("JDy", C.c_void_p), ("JDz", C.c_void_p),
                ("psi", C.c_void_p), ("mat", C.c_void_p), ("dft", C.c_void_p)]


class cpl_desc(C.Structure):
    _fields_ = [("qd", qd_desc), ("fd", fdtd_desc), ("n_occ", C.c_int32),
                ("mol_weight", C.c_double), ("mol_every", C.c_int32),
                ("held_k0", C.c_int32), ("held_nk", C.c_int32)]


class cpl_state(C.Structure):
    _fields_ = [("psi", C.c_void_p), ("absorbed", C.c_void_p), ("d_mol", C.c_void_p),
                ("E_mol", C.c_void_p), ("P_c", C.c_void_p), ("J_mol", C.c_void_p),
                ("cell_of_mol", C.c_void_p), ("occ_cell", C.c_void_p), ("occ_ptr", C.c_void_p),
                ("mol_perm", C.c_void_p), ("f", fdtd_fields), ("qd_ws", C.c_void_p),
                ("fd_ws", C.c_void_p), ("psi_next", C.c_void_p), ("E_held", C.c_void_p)]


class bloch_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("prec", C.c_int32), ("omega0_au", C.c_double),
                ("mu_au", C.c_double), ("gamma1_au", C.c_double), ("gamma2_au", C.c_double),
                ("dt_au", C.c_double)]


class cpl_bloch_desc(C.Structure):
    _fields_ = [("bl", bloch_desc), ("fd", fdtd_desc), ("n_occ", C.c_int32), ("weight", C.c_double)]


class cpl_bloch_state(C.Structure):
    _fields_ = [("state", C.c_void_p), ("d_mol", C.c_void_p), ("E_mol", C.c_void_p),
                ("P_c", C.c_void_p), ("J_mol", C.c_void_p), ("cell_of_mol", C.c_void_p),
                ("occ_cell", C.c_void_p), ("occ_ptr", C.c_void_p), ("mol_perm", C.c_void_p),
                ("f", fdtd_fields), ("fd_ws", C.c_void_p)]


class cpl_adj(C.Structure):
    _fields_ = [("lpsi", C.c_void_p), ("labs", C.c_void_p), ("lP", C.c_void_p), ("ld", C.c_void_p),
                ("lE", C.c_void_p), ("lf", fdtd_fields), ("scratch", C.c_void_p), ("lJ", C.c_void_p)]


_vp, _dp, _i32p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
_sigs = {
    "msqd_last_error": (C.c_char_p, []),
    "msqd_version": (C.c_int, []),
    "msqd_mol_timing_begin": (C.c_int, [C.c_int32]),
    "msqd_mol_timing_end": (C.c_int, [_dp, _i32p]),
    "qd_workspace_bytes": (C.c_size_t, [C.POINTER(qd_desc)]),
    "qd_init": (C.c_int, [C.POINTER(qd_desc), _dp, _dp, _dp, _dp, _vp, C.c_size_t, _vp, _vp, _vp]),
    "qd_step": (C.c_int, [C.POINTER(qd_desc), _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp]),
    "dipole_readout": (C.c_int, [C.POINTER(qd_desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "dipole_readout_noalloc": (C.c_int, [C.POINTER(qd_desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "msqd_check_status": (C.c_int, [_vp, _vp]),
    "qd_jm_tables_size": (C.c_size_t, [C.c_int32]),
    "qd_jm_tables": (C.c_int, [C.c_int32, _dp, C.c_size_t]),
    "fdtd_workspace_bytes": (C.c_size_t, [C.POINTER(fdtd_desc)]),
    "fdtd_psi_bytes": (C.c_size_t, [C.POINTER(fdtd_desc)]),
    "fdtd_dft_bytes": (C.c_size_t, [C.POINTER(fdtd_desc)]),
    "fdtd_init": (C.c_int, [C.POINTER(fdtd_desc), _vp, _dp, C.POINTER(fdtd_fields), _vp,
                            C.c_size_t, _vp]),
    "fdtd_step": (C.c_int, [C.POINTER(fdtd_desc), C.POINTER(fdtd_fields), _vp, C.c_int64,
                            C.c_double, _vp]),
    "flux_readout": (C.c_int, [C.POINTER(fdtd_desc), C.POINTER(fdtd_fields), _vp, _vp]),
    "spectra_readout": (C.c_int, [C.POINTER(fdtd_desc), _vp, _vp, _vp, _vp]),
    "map_build": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_int32,
                            C.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p]),
    "map_csr": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p]),
    "map_planes": (C.c_int, [C.c_int32, _i32p, C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p]),
    "coupled_step": (C.c_int, [C.POINTER(cpl_desc), C.POINTER(cpl_state), _dp, C.c_int64,
                               C.c_int32, _vp]),
    "adjoint_scratch_bytes": (C.c_size_t, [C.POINTER(cpl_desc)]),
    "adjoint_init_yield": (C.c_int, [C.POINTER(cpl_desc), C.POINTER(cpl_state), C.POINTER(cpl_adj),
                                     _vp]),
    "adjoint_step": (C.c_int, [C.POINTER(cpl_desc), C.POINTER(cpl_state), _vp, _vp, _vp,
                               C.POINTER(cpl_adj), C.c_int64, _vp, _vp]),
    "excited_r_readout": (C.c_int, [C.POINTER(qd_desc), _vp, _vp, _vp, _vp, _vp, _vp]),
    "bloch_init": (C.c_int, [C.POINTER(bloch_desc), _vp, _vp]),
    "bloch_step": (C.c_int, [C.POINTER(bloch_desc), _vp, _vp, _vp, C.c_int32, _vp]),
    "coupled_bloch_step": (C.c_int, [C.POINTER(cpl_bloch_desc), C.POINTER(cpl_bloch_state), _dp,
                                     C.c_int64, C.c_int32, _vp]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def last_error() -> str:
    return lib.msqd_last_error().decode()


def _check(rc):
    if rc != MSQD_OK:
        raise MsqdError(rc, last_error())
    return rc


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return C.c_void_p(t.data_ptr())
    return t


def _np_dp(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def current_stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# --------------------------------------------------------------- raw calls
def qd_workspace_bytes(d: qd_desc) -> int:
    n = lib.qd_workspace_bytes(C.byref(d))
    if n == 0:
        raise MsqdError(MSQD_EINVAL, last_error())
    return n


def qd_init(d, U_g, U_e, mu12, psi0, ws, psi, absorbed, stream=None):
    ug, pug = _np_dp(U_g)
    ue, pue = _np_dp(U_e)
    mu, pmu = _np_dp(mu12)
    p0, pp0 = _np_dp(psi0)
    return _check(lib.qd_init(C.byref(d), pug, pue, pmu, pp0, _ptr(ws), ws.numel() * ws.element_size(),
                              _ptr(psi), _ptr(absorbed), stream or current_stream()))


def qd_step(d, ws, psi, E_mol, absorbed, d_mol=None, n_steps=1, stream=None):
    return _check(lib.qd_step(C.byref(d), _ptr(ws), _ptr(psi), _ptr(E_mol), _ptr(absorbed),
                              _ptr(d_mol), int(n_steps), stream or current_stream()))


def dipole_readout(d, ws, psi, absorbed, d_mol=None, norm_mol=None, yield_mol=None, sums=None,
                   stream=None):
    return _check(lib.dipole_readout(C.byref(d), _ptr(ws), _ptr(psi), _ptr(absorbed), _ptr(d_mol),
                                     _ptr(norm_mol), _ptr(yield_mol), _ptr(sums),
                                     stream or current_stream()))


def dipole_readout_noalloc(d, ws, psi, absorbed, d_mol=None, norm_mol=None, yield_mol=None, sums=None,
                           stream=None):
    return _check(lib.dipole_readout_noalloc(C.byref(d), _ptr(ws), _ptr(psi), _ptr(absorbed), _ptr(d_mol),
                                             _ptr(norm_mol), _ptr(yield_mol), _ptr(sums),
                                             stream or current_stream()))


def jm_tables(j_max):
    """The host-built tables of the general (j, m) coupling (2 <= j_max <= 5)
    as a float64 array, in the layout include/msqd.h documents for
    qd_jm_tables."""
    n = lib.qd_jm_tables_size(int(j_max))
    out = np.zeros(max(n, 1), dtype=np.float64)
    _check(lib.qd_jm_tables(int(j_max), out.ctypes.data_as(_dp), n))
    return out[:n]


def mol_timing_begin(max_launches):
    """Start recording HIP events around the molecular-step launches of
    coupled_step on this thread (instrumentation only)."""
    return _check(lib.msqd_mol_timing_begin(int(max_launches)))


def mol_timing_end():
    """(summed ms, launches) of the molecular-step launches recorded since
    mol_timing_begin; waits for their events."""
    ms = C.c_double(0.0)
    n = C.c_int32(0)
    _check(lib.msqd_mol_timing_end(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def check_status(ws, stream=None):
    return _check(lib.msqd_check_status(_ptr(ws), stream or current_stream()))


def fdtd_init(d, mat_host, freqs, f, ws, stream=None):
    mat = np.ascontiguousarray(mat_host, dtype=np.uint8)
    fr, pfr = _np_dp(freqs if freqs is not None and len(freqs) else np.zeros(1))
    return _check(lib.fdtd_init(C.byref(d), mat.ctypes.data_as(C.c_void_p), pfr, C.byref(f),
                                _ptr(ws), ws.numel() * ws.element_size(),
                                stream or current_stream()))


def fdtd_step(d, f, ws, n, src_value, stream=None):
    return _check(lib.fdtd_step(C.byref(d), C.byref(f), _ptr(ws), int(n), float(src_value),
                                stream or current_stream()))


def flux_readout(d, f, flux, stream=None):
    return _check(lib.flux_readout(C.byref(d), C.byref(f), _ptr(flux), stream or current_stream()))


def spectra_readout(d, flux, flux_ref, tra, stream=None):
    return _check(lib.spectra_readout(C.byref(d), _ptr(flux), _ptr(flux_ref), _ptr(tra),
                                      stream or current_stream()))


def map_build(n_mol, nx, ny, nz, seed, slab_k0, slab_nk):
    """Host call: returns (cell_of_mol, occ_cell, occ_ptr, mol_perm) int32 arrays."""
    cell = np.zeros(n_mol, np.int32)
    occ = np.zeros(max(n_mol, 1), np.int32)
    ptr = np.zeros(n_mol + 1, np.int32)
    perm = np.zeros(max(n_mol, 1), np.int32)
    n_occ = C.c_int32(0)
    _check(lib.map_build(n_mol, nx, ny, nz, C.c_uint64(seed), slab_k0, slab_nk,
                         cell.ctypes.data_as(_i32p), occ.ctypes.data_as(_i32p),
                         ptr.ctypes.data_as(_i32p), perm.ctypes.data_as(_i32p), C.byref(n_occ)))
    k = n_occ.value
    return cell, occ[:k].copy(), ptr[:k + 1].copy(), perm[:n_mol].copy()


def map_csr(cell_of_mol, n_cells):
    cell = np.ascontiguousarray(cell_of_mol, dtype=np.int32)
    n_mol = len(cell)
    occ = np.zeros(max(n_mol, 1), np.int32)
    ptr = np.zeros(n_mol + 1, np.int32)
    perm = np.zeros(max(n_mol, 1), np.int32)
    n_occ = C.c_int32(0)
    _check(lib.map_csr(n_mol, n_cells, cell.ctypes.data_as(_i32p), occ.ctypes.data_as(_i32p),
                       ptr.ctypes.data_as(_i32p), perm.ctypes.data_as(_i32p), C.byref(n_occ)))
    k = n_occ.value
    return occ[:k].copy(), ptr[:k + 1].copy(), perm[:n_mol].copy()


def map_planes(occ_cell, nx, ny, nz):
    """(held_k0, held_nk): the planes that hold every occupied cell."""
    occ = np.ascontiguousarray(occ_cell, dtype=np.int32)
    k0, nk = C.c_int32(0), C.c_int32(0)
    _check(lib.map_planes(len(occ), occ.ctypes.data_as(_i32p), nx, ny, nz, C.byref(k0), C.byref(nk)))
    return k0.value, nk.value


def coupled_step(d, st, src_values, n0, stream=None):
    src, psrc = _np_dp(src_values)
    return _check(lib.coupled_step(C.byref(d), C.byref(st), psrc, int(n0), len(src),
                                   stream or current_stream()))


def adjoint_init_yield(d, st, adj, stream=None):
    return _check(lib.adjoint_init_yield(C.byref(d), C.byref(st), C.byref(adj),
                                         stream or current_stream()))


def adjoint_step(d, st, psi_n, E_mol_n, adj, n, g_src, psi_np1=None, stream=None):
    return _check(lib.adjoint_step(C.byref(d), C.byref(st), _ptr(psi_n), _ptr(psi_np1), _ptr(E_mol_n),
                                   C.byref(adj), int(n), _ptr(g_src), stream or current_stream()))


# ------------------------------------------------------------ allocations
def _dev():
    return torch.device("cuda", torch.cuda.current_device())


class Molecules:
    """Wavepacket batch: descriptor, workspace, psi, absorbed, readout buffers."""

    def __init__(self, n_mol, n_r, j_max, r_min, r_max, mass, dt_au, U_g, U_e, mu12, psi0,
                 prec="fp64", absorb_width=2.0, r_diss=8.0, basis="m0"):
        self.prec = PREC[prec] if isinstance(prec, str) else prec
        self.basis = BASIS[basis] if isinstance(basis, str) else basis
        self.desc = qd_desc(int(n_mol), int(n_r), int(j_max), self.prec, float(r_min), float(r_max),
                            float(mass), float(dt_au), float(absorb_width), float(r_diss), self.basis)
        dev = _dev()
        nbytes = qd_workspace_bytes(self.desc)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        cdt = torch.complex128 if self.prec == FP64 else torch.complex64
        nj = int(j_max) + 1
        self.n_ang = nj * nj if self.basis == BASIS_JM else nj     # lines per electronic state
        self.psi = torch.empty((int(n_mol), 2, self.n_ang, int(n_r)), dtype=cdt, device=dev)
        self.absorbed = torch.zeros(int(n_mol), dtype=torch.float64, device=dev)
        dshape = (int(n_mol), 3) if self.basis == BASIS_JM else (int(n_mol),)
        self.d = torch.zeros(dshape, dtype=torch.float64, device=dev)
        qd_init(self.desc, U_g, U_e, mu12, psi0, self.ws, self.psi, self.absorbed)

    @classmethod
    def from_config(cls, cfg, n_mol=None, prec=None, dt_au=None):
        from workloads.molecule_inputs import morse_v0, potentials
        ug, ue, mu = potentials(cfg)
        return cls(cfg.n_mol if n_mol is None else n_mol, cfg.n_r, cfg.j_max, cfg.r_min, cfg.r_max,
                   cfg.mass, cfg.dt_au if dt_au is None else dt_au, ug, ue, mu, morse_v0(cfg),
                   prec or cfg.precision, cfg.absorb_width, cfg.r_diss, cfg.basis)

    def step(self, E_mol, n_steps=1, want_d=True):
        qd_step(self.desc, self.ws, self.psi, E_mol, self.absorbed, self.d if want_d else None,
                n_steps)

    @property
    def n_sums(self):
        """Entries of dipole_readout's ensemble sums: the dipole components
        (1, or x, y, z in the (j, m) basis), then the norm and the yield."""
        return (3 if self.basis == BASIS_JM else 1) + 2

    def readout(self, sums=None):
        """Per-molecule (d, norm, yield) of the current state; with `sums` (a
        device float64 tensor of n_sums entries, or a row of a larger one)
        also their fixed-order ensemble sums."""
        n = self.desc.n_mol
        dev = self.psi.device
        d = torch.empty((max(n, 1),) + tuple(self.d.shape[1:]), dtype=torch.float64, device=dev)
        nrm = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        yld = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
        dipole_readout(self.desc, self.ws, self.psi, self.absorbed, d, nrm, yld, sums)
        return d, nrm, yld

    def ensemble_sums(self, out=None):
        """Device float64 [n_sums]: sum of the dipoles, of the norms and of
        the yields over the batch (dipole_readout's sums), written into `out`
        when given."""
        if out is None:
            out = torch.empty(self.n_sums, dtype=torch.float64, device=self.psi.device)
        if not hasattr(self, "_rd_buf"):       # per-molecule outputs the sums reduce, kept for reuse
            n = max(self.desc.n_mol, 1)
            self._rd_buf = (torch.empty((n,) + tuple(self.d.shape[1:]), dtype=torch.float64,
                                        device=self.psi.device),
                            torch.empty(n, dtype=torch.float64, device=self.psi.device),
                            torch.empty(n, dtype=torch.float64, device=self.psi.device))
        d, nrm, yld = self._rd_buf
        dipole_readout(self.desc, self.ws, self.psi, self.absorbed, d, nrm, yld, out)
        return out


def excited_r(mols):
    """Eq. (8) readout of a Molecules batch: (per-molecule <R>_e numerators,
    excited populations, ensemble <R>_e) as device tensors.  The ensemble
    value is the library's ratio of the two ensemble sums, so it is NaN while
    the excited population is exactly zero."""
    n = max(mols.desc.n_mol, 1)
    dev = mols.psi.device
    num = torch.empty(n, dtype=torch.float64, device=dev)
    pop = torch.empty(n, dtype=torch.float64, device=dev)
    sums = torch.empty(3, dtype=torch.float64, device=dev)
    _check(lib.excited_r_readout(C.byref(mols.desc), _ptr(mols.ws), _ptr(mols.psi), _ptr(num),
                                 _ptr(pop), _ptr(sums), current_stream()))
    return num, pop, sums[2]


def spectra(fields, flux, flux_ref):
    """(T, R, A) device tensors per monitor frequency (spectra_readout): flux
    is the [2, n_freq] readout of a run with both detection planes, flux_ref
    the [n_freq] incident-side flux of a reference run without the
    structure."""
    tra = torch.empty((3, fields.desc.n_freq), dtype=torch.float64, device=flux.device)
    spectra_readout(fields.desc, flux.contiguous(), flux_ref.contiguous(), tra)
    return tra[0], tra[1], tra[2]


def fdtd_desc_from_config(cfg, prec=None, n_freq=None):
    from workloads.geometry import eps_table
    p = PREC[prec or cfg.precision]
    eps = eps_table(cfg)
    nf = cfg.n_freq if n_freq is None else n_freq
    return fdtd_desc(cfg.nx, cfg.ny, cfg.nz, cfg.npml, p, 2, cfg.dx, cfg.dt,
                     (C.c_double * 4)(eps[0], eps[1], eps[2], 1.0), cfg.wp, cfg.gamma, cfg.cpml_m,
                     cfg.sigma_max_lo, cfg.sigma_max_hi, cfg.cpml_kappa_max, cfg.cpml_alpha_max,
                     cfg.src_k, cfg.mon_k, nf, cfg.mon_every, cfg.mon_k2)


class Fields:
    """Yee field buffers (torch) plus the descriptor and workspace."""

    def __init__(self, desc: fdtd_desc, mat_host, freqs):
        self.desc = desc
        dev = _dev()
        dt = torch.float64 if desc.prec == FP64 else torch.float32
        shape = (desc.nz, desc.ny, desc.nx)
        names = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "JDx", "JDy", "JDz"]
        self.t = {n: torch.empty(shape, dtype=dt, device=dev) for n in names}
        psi_bytes = lib.fdtd_psi_bytes(C.byref(desc))
        self.t["psi"] = torch.empty(max(psi_bytes // (8 if desc.prec == FP64 else 4), 1), dtype=dt,
                                    device=dev)
        self.t["mat"] = torch.empty((3,) + shape, dtype=torch.uint8, device=dev)
        dft_bytes = lib.fdtd_dft_bytes(C.byref(desc))
        self.t["dft"] = torch.empty(max(dft_bytes // 16, 1), dtype=torch.complex128, device=dev)
        nbytes = lib.fdtd_workspace_bytes(C.byref(desc))
        if nbytes == 0:
            raise MsqdError(MSQD_EINVAL, last_error())
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.f = fdtd_fields(*[C.c_void_p(self.t[n].data_ptr()) for n in names + ["psi", "mat"]],
                             C.c_void_p(self.t["dft"].data_ptr()) if desc.n_freq > 0 else None)
        fdtd_init(desc, mat_host, freqs, self.f, self.ws)

    def __getattr__(self, name):
        t = self.__dict__.get("t")
        if t is not None and name in t:
            return t[name]
        raise AttributeError(name)

    def step(self, n, src_value):
        fdtd_step(self.desc, self.f, self.ws, n, src_value)

    @property
    def n_planes(self):
        return 2 if (self.desc.n_freq > 0 and self.desc.mon_k2 != 0) else 1

    def flux(self):
        """Net z-flux per monitor frequency on the mon_k plane, or
        [2, n_freq] (mon_k, then mon_k2) when the second plane is set."""
        nf = self.desc.n_freq
        out = torch.zeros(self.n_planes * nf, dtype=torch.float64, device=self.ws.device)
        flux_readout(self.desc, self.f, out)
        return out if self.n_planes == 1 else out.view(2, nf)

    def dft_planes(self):
        nf, ny, nx = self.desc.n_freq, self.desc.ny, self.desc.nx
        return self.t["dft"][: 4 * nf * ny * nx].view(4, nf, ny, nx)


class Coupled:
    """The self-consistent system: molecules + fields + maps, driven by
    coupled_step."""

    def __init__(self, cfg, prec=None, n_mol=None, cells=None, mat=None, n_freq=None, mol_every=1,
                 held=True):
        """held: let the E update subtract the molecular current from an
        array over the planes of the occupied cells (coupled_step's E_held),
        instead of a separate pass after it; the results are the same."""
        from workloads.geometry import material_map
        prec = prec or cfg.precision
        self.cfg = cfg
        dev = _dev()
        if mat is None:
            mat = material_map(cfg)
        self.fields = Fields(fdtd_desc_from_config(cfg, prec, n_freq), mat, cfg.freqs)
        if cells is None:
            if cfg.placement == "block":
                from workloads.molecule_inputs import block_cell_list
                cells = block_cell_list(cfg)
                occ, ptr, perm = map_csr(cells, cfg.nx * cfg.ny * cfg.nz)
            else:
                cells, occ, ptr, perm = map_build(cfg.n_mol, cfg.nx, cfg.ny, cfg.nz, cfg.seed,
                                                  cfg.slab_k0, cfg.slab_nk)
        else:
            cells = np.asarray(cells, np.int32)
            occ, ptr, perm = map_csr(cells, cfg.nx * cfg.ny * cfg.nz)
        if n_mol is not None and n_mol != len(cells):
            cells = cells[:n_mol]
            occ, ptr, perm = map_csr(cells, cfg.nx * cfg.ny * cfg.nz)
        self.cells_host = cells
        self.mol_every = max(1, int(mol_every))
        self.mol = Molecules.from_config(cfg, n_mol=len(cells), prec=prec,
                                         dt_au=cfg.dt_au * self.mol_every)
        it = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32), device=dev)  # noqa: E731
        self.cell_of_mol = it(cells)
        self.occ_cell = it(occ)
        self.occ_ptr = it(ptr)
        self.mol_perm = it(perm)
        nm = len(cells)
        nc = 3 if self.mol.basis == BASIS_JM else 1       # field components coupled
        shp = (lambda n: (max(n, 1), 3)) if nc == 3 else (lambda n: (max(n, 1),))  # noqa: E731
        self.E_mol = torch.zeros(shp(nm), dtype=torch.float64, device=dev)
        self.P_c = torch.zeros(shp(len(occ)), dtype=torch.float64, device=dev)
        self.J_mol = torch.zeros(shp(len(occ)), dtype=torch.float64, device=dev)
        self.desc = cpl_desc(self.mol.desc, self.fields.desc, len(occ), float(cfg.mol_weight),
                             self.mol_every)
        self.state = cpl_state(C.c_void_p(self.mol.psi.data_ptr()),
                               C.c_void_p(self.mol.absorbed.data_ptr()),
                               C.c_void_p(self.mol.d.data_ptr()), C.c_void_p(self.E_mol.data_ptr()),
                               C.c_void_p(self.P_c.data_ptr()), C.c_void_p(self.J_mol.data_ptr()),
                               C.c_void_p(self.cell_of_mol.data_ptr()),
                               C.c_void_p(self.occ_cell.data_ptr()),
                               C.c_void_p(self.occ_ptr.data_ptr()),
                               C.c_void_p(self.mol_perm.data_ptr()), self.fields.f,
                               C.c_void_p(self.mol.ws.data_ptr()),
                               C.c_void_p(self.fields.ws.data_ptr()))
        self.E_held = None
        if held and len(occ) > 0:
            k0, nk = map_planes(occ, cfg.nx, cfg.ny, cfg.nz)
            self.desc.held_k0, self.desc.held_nk = k0, nk
            self.E_held = torch.zeros((nc, nk, cfg.ny, cfg.nx), dtype=self.fields.t["Ex"].dtype, device=dev)
            self.state.E_held = C.c_void_p(self.E_held.data_ptr())
        self.n = 0

    def step(self, src_values):
        src_values = np.atleast_1d(np.asarray(src_values, np.float64))
        coupled_step(self.desc, self.state, src_values, self.n)
        self.n += len(src_values)

    def step_out_of_place(self, src_value, psi_in, psi_out, E_out=None):
        """One coupled step whose molecules read psi_in and write the stepped
        wavepackets to psi_out (coupled_step's psi_next); the fields, the
        absorbed norms and the polarisation advance as in step().  E_out:
        where the molecular step records the field it gathered (float64
        [n_mol]) instead of self.E_mol."""
        src_values = np.atleast_1d(np.asarray(src_value, np.float64))
        self.state.psi = C.c_void_p(psi_in.data_ptr())
        self.state.psi_next = C.c_void_p(psi_out.data_ptr())
        if E_out is not None:
            self.state.E_mol = C.c_void_p(E_out.data_ptr())
        try:
            coupled_step(self.desc, self.state, src_values, self.n)
        finally:
            self.state.psi = C.c_void_p(self.mol.psi.data_ptr())
            self.state.psi_next = None
            self.state.E_mol = C.c_void_p(self.E_mol.data_ptr())
        self.n += 1

    # -------------------------------------------------- checkpoint / restore
    _STATE = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "JDx", "JDy", "JDz", "psi", "dft"]

    def snapshot(self):
        """Device copy of everything a later step reads (checkpoint)."""
        snap = {k: self.fields.t[k].clone() for k in self._STATE}
        snap["mol_psi"] = self.mol.psi.clone()
        snap["absorbed"] = self.mol.absorbed.clone()
        snap["P_c"] = self.P_c.clone()
        snap["J_mol"] = self.J_mol.clone()
        snap["n"] = self.n
        return snap

    def restore(self, snap):
        for k in self._STATE:
            self.fields.t[k].copy_(snap[k])
        self.mol.psi.copy_(snap["mol_psi"])
        self.mol.absorbed.copy_(snap["absorbed"])
        self.P_c.copy_(snap["P_c"])
        self.J_mol.copy_(snap["J_mol"])
        self.n = snap["n"]

    def ensemble_sums(self, out=None):
        """dipole_readout's ensemble sums of the current state (device
        float64: the dipole components, then the norm and the yield)."""
        return self.mol.ensemble_sums(out)

    def adjoint_buffers(self):
        """Allocate the adjoint state (same shapes as the forward state)."""
        dev = self.mol.psi.device
        fd = self.fields
        t = {n: torch.zeros_like(fd.t[n]) for n in ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz",
                                                      "JDx", "JDy", "JDz", "psi"]}
        t["lpsi"] = torch.zeros_like(self.mol.psi)
        nm = max(self.mol.desc.n_mol, 1)
        t["labs"] = torch.zeros(nm, dtype=torch.float64, device=dev)
        t["ld"] = torch.zeros(nm, dtype=torch.float64, device=dev)
        t["lE"] = torch.zeros(nm, dtype=torch.float64, device=dev)
        t["lP"] = torch.zeros(max(self.desc.n_occ, 1), dtype=torch.float64, device=dev)
        t["lJ"] = torch.zeros(max(self.desc.n_occ, 1), dtype=torch.float64, device=dev)
        nbytes = lib.adjoint_scratch_bytes(C.byref(self.desc))
        t["scratch"] = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=dev)
        lf = fdtd_fields(*[C.c_void_p(t[n].data_ptr()) for n in ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz",
                                                                  "JDx", "JDy", "JDz", "psi"]],
                         None, None)
        adj = cpl_adj(C.c_void_p(t["lpsi"].data_ptr()), C.c_void_p(t["labs"].data_ptr()),
                      C.c_void_p(t["lP"].data_ptr()), C.c_void_p(t["ld"].data_ptr()),
                      C.c_void_p(t["lE"].data_ptr()), lf, C.c_void_p(t["scratch"].data_ptr()),
                      C.c_void_p(t["lJ"].data_ptr()))
        return adj, t


class Bloch:
    """Frozen two-level emitters: descriptor and the [3][n] state planes."""

    def __init__(self, n, omega0, mu, dt_au, prec="fp64", gamma1=0.0, gamma2=0.0):
        self.prec = PREC[prec] if isinstance(prec, str) else prec
        self.desc = bloch_desc(int(n), self.prec, float(omega0), float(mu), float(gamma1),
                               float(gamma2), float(dt_au))
        dt = torch.float64 if self.prec == FP64 else torch.float32
        self.state = torch.empty((3, max(int(n), 1)), dtype=dt, device=_dev())
        self.d = torch.zeros(max(int(n), 1), dtype=torch.float64, device=_dev())
        _check(lib.bloch_init(C.byref(self.desc), _ptr(self.state), current_stream()))

    @classmethod
    def from_config(cls, cfg, n=None, prec=None, dt_au=None):
        from workloads.molecule_inputs import bloch_parameters
        w0, mu = bloch_parameters(cfg)
        return cls(cfg.n_mol if n is None else n, w0, mu, cfg.dt_au if dt_au is None else dt_au,
                   prec or cfg.precision)

    def step(self, E, n_steps=1):
        _check(lib.bloch_step(C.byref(self.desc), _ptr(self.state), _ptr(E), _ptr(self.d),
                              int(n_steps), current_stream()))


class CoupledBloch:
    """The coupled system with Bloch emitters in place of the wavepackets."""

    def __init__(self, cfg, prec=None, model=None, cells=None, mat=None, n_freq=None):
        from workloads.geometry import material_map
        prec = prec or cfg.precision
        self.cfg = cfg
        dev = _dev()
        if mat is None:
            mat = material_map(cfg)
        self.fields = Fields(fdtd_desc_from_config(cfg, prec, n_freq), mat, cfg.freqs)
        if cells is None:
            if cfg.placement == "block":
                from workloads.molecule_inputs import block_cell_list
                cells = block_cell_list(cfg)
                occ, ptr, perm = map_csr(cells, cfg.nx * cfg.ny * cfg.nz)
            else:
                cells, occ, ptr, perm = map_build(cfg.n_mol, cfg.nx, cfg.ny, cfg.nz, cfg.seed,
                                                  cfg.slab_k0, cfg.slab_nk)
        else:
            cells = np.asarray(cells, np.int32)
            occ, ptr, perm = map_csr(cells, cfg.nx * cfg.ny * cfg.nz)
        n = len(cells)
        if model is None:
            self.em = Bloch.from_config(cfg, n=n, prec=prec)
        else:
            w0, mu = model
            self.em = Bloch(n, w0, mu, cfg.dt_au, prec)
        it = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32), device=dev)  # noqa: E731
        self.cell_of_mol, self.occ_cell, self.occ_ptr, self.mol_perm = it(cells), it(occ), it(ptr), it(perm)
        self.E_mol = torch.zeros(max(n, 1), dtype=torch.float64, device=dev)
        self.P_c = torch.zeros(max(len(occ), 1), dtype=torch.float64, device=dev)
        self.J_mol = torch.zeros(max(len(occ), 1), dtype=torch.float64, device=dev)
        self.desc = cpl_bloch_desc(self.em.desc, self.fields.desc, len(occ), float(cfg.mol_weight))
        self.state = cpl_bloch_state(_ptr(self.em.state), _ptr(self.em.d), _ptr(self.E_mol),
                                     _ptr(self.P_c), _ptr(self.J_mol), _ptr(self.cell_of_mol),
                                     _ptr(self.occ_cell), _ptr(self.occ_ptr), _ptr(self.mol_perm),
                                     self.fields.f, _ptr(self.fields.ws))
        self.n = 0

    def step(self, src_values):
        src, psrc = _np_dp(np.atleast_1d(src_values))
        _check(lib.coupled_bloch_step(C.byref(self.desc), C.byref(self.state), psrc, self.n, len(src),
                                      current_stream()))
        self.n += len(src_values)


class CarrierBatch:
    """Several independent coupled runs (one per incident carrier, the
    paper's frequency scans) advanced together: each run has its own state
    and its own stream, and the runs' launches are interleaved step by step
    so that the GPU overlaps one run's small field kernels with another's
    molecular step.  Every run computes exactly what it computes alone."""

    def __init__(self, cfgs, prec=None, **kw):
        self.systems = [Coupled(c, prec=prec, **kw) for c in cfgs]
        self.streams = [torch.cuda.Stream() for _ in cfgs]   # default priority
        torch.cuda.synchronize()

    def step(self, src_values_per_run, chunk=1):
        """src_values_per_run: one array of source samples per run (same
        length); advances every run by that many steps."""
        n = len(src_values_per_run[0])
        for t in range(0, n, chunk):
            for sysm, st, src in zip(self.systems, self.streams, src_values_per_run):
                with torch.cuda.stream(st):
                    sysm.step(src[t:t + chunk])

    def synchronize(self):
        for st in self.streams:
            st.synchronize()


def n_exports_ok():
    return all(hasattr(lib, n) for n in EXPORTS)


def version():
    return lib.msqd_version()


__all__ = ["Molecules", "Fields", "Coupled", "Bloch", "CoupledBloch", "CarrierBatch", "qd_init", "qd_step",
           "dipole_readout", "fdtd_init", "fdtd_step", "flux_readout", "spectra_readout", "spectra",
           "excited_r", "map_build", "map_csr", "map_planes", "coupled_step", "check_status", "jm_tables", "MsqdError", "lib",
           "LIB_PATH", "EXPORTS"]
