"""The C-ABI library: it loads without a GPU, exports every declared symbol,
validates descriptors on the host, and its host-side map builder matches the
oracle bit for bit.  No compute call touches a device here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msqd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def msqd():
    from paper_2209_04487_amd import msqd as m
    return m


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["qd_init", "qd_step", "fdtd_step", "coupled_step", "dipole_readout",
                     "map_build", "fdtd_init", "flux_readout", "msqd_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(msqd):
    for name in _declared_functions():
        assert hasattr(msqd.lib, name), name


def test_workspace_queries_and_validation(msqd):
    d = msqd.qd_desc(10, 256, 10, msqd.FP64, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, 0)
    assert msqd.lib.qd_workspace_bytes(C.byref(d)) > 0
    # dipole_readout's partial sums grow with the batch: 3 doubles per block of 1024 molecules
    grow = msqd.qd_desc(10 + 3 * 1024, 256, 10, msqd.FP64, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, 0)
    assert msqd.lib.qd_workspace_bytes(C.byref(grow)) == msqd.lib.qd_workspace_bytes(C.byref(d)) + 3 * 3 * 8
    bad = msqd.qd_desc(10, 100, 10, msqd.FP64, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, 0)
    assert msqd.lib.qd_workspace_bytes(C.byref(bad)) == 0
    assert "n_r" in msqd.last_error()
    bad = msqd.qd_desc(10, 256, 16, msqd.FP64, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0)
    assert msqd.lib.qd_workspace_bytes(C.byref(bad)) == 0
    bad = msqd.qd_desc(10, 256, 10, 7, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0)
    assert msqd.lib.qd_workspace_bytes(C.byref(bad)) == 0
    # qd_init rejects before touching the device
    rc = msqd.lib.qd_init(C.byref(bad), None, None, None, None, None, 0, None, None, None)
    assert rc == msqd.MSQD_EPREC


def test_fdtd_validation(msqd):
    from workloads import get_config
    cfg = get_config("cfg0")
    d = msqd.fdtd_desc_from_config(cfg)
    assert msqd.lib.fdtd_workspace_bytes(C.byref(d)) > 0
    d.dt = d.dt * 2.0  # Courant 1.0 > 1/sqrt(3)
    assert msqd.lib.fdtd_workspace_bytes(C.byref(d)) == 0
    assert "Courant" in msqd.last_error()
    d = msqd.fdtd_desc_from_config(cfg)
    d.mon_k = 2   # inside the CPML
    assert msqd.lib.fdtd_workspace_bytes(C.byref(d)) == 0
    rc = msqd.lib.fdtd_step(C.byref(d), None, None, 0, 0.0, None)
    assert rc == msqd.MSQD_EINVAL
    d = msqd.fdtd_desc_from_config(cfg)
    d.nx, d.ny, d.nz = 1, 1, 70000   # one launch row holds at most 65535 planes
    assert msqd.lib.fdtd_workspace_bytes(C.byref(d)) == 0
    assert "65535" in msqd.last_error()
    d = msqd.fdtd_desc_from_config(cfg)
    d.n_freq = 70000
    assert msqd.lib.fdtd_workspace_bytes(C.byref(d)) == 0
    assert "n_freq" in msqd.last_error()


@pytest.mark.parametrize("cfgname", ["cfg1", "cfg3"])
def test_map_build_bit_exact_with_oracle(msqd, cfgname):
    from oracle.maps import csr, slab_cells
    from workloads import get_config
    cfg = get_config(cfgname)
    n = 20000 if cfgname == "cfg1" else cfg.n_mol
    cell, occ, ptr, perm = msqd.map_build(n, cfg.nx, cfg.ny, cfg.nz, cfg.seed, cfg.slab_k0,
                                          cfg.slab_nk)
    oc = slab_cells(cfg.seed, n, cfg.nx, cfg.ny, cfg.slab_k0, cfg.slab_nk)
    oo, op, om = csr(oc)
    assert np.array_equal(cell, oc)
    assert np.array_equal(occ, oo)
    assert np.array_equal(ptr, op)
    assert np.array_equal(perm, om)


def test_map_edge_cases(msqd):
    cell, occ, ptr, perm = msqd.map_build(0, 8, 8, 8, 1, 2, 2)
    assert len(cell) == 0 and len(occ) == 0 and list(ptr) == [0]
    cell, occ, ptr, perm = msqd.map_build(1, 1, 1, 8, 1, 3, 1)
    assert list(cell) == [3] and list(occ) == [3] and list(ptr) == [0, 1]
    with pytest.raises(msqd.MsqdError):
        msqd.map_build(10, 8, 8, 8, 1, 6, 4)   # slab beyond the grid
    with pytest.raises(msqd.MsqdError):
        msqd.map_csr(np.array([0, 5, 64]), 64)  # index out of range
    occ, ptr, perm = msqd.map_csr(np.array([5, 2, 5, 5, 2]), 64)
    assert list(occ) == [2, 5] and list(ptr) == [0, 2, 5] and list(perm) == [1, 4, 0, 2, 3]


def test_coupled_step_checks_multirate_step(msqd):
    """coupled_step validates on the host, before any launch: the molecular
    step must be mol_every field steps (here 4 dt against mol_every = 5), and
    a negative mol_every is rejected.  The device pointers are never touched
    (placeholder aligned addresses)."""
    from workloads import get_config
    cfg = get_config("cfg0")
    qd = msqd.qd_desc(64, cfg.n_r, cfg.j_max, msqd.FP64, cfg.r_min, cfg.r_max, cfg.mass,
                      cfg.dt_au * 4, cfg.absorb_width, cfg.r_diss)
    fd = msqd.fdtd_desc_from_config(cfg, "fp64")
    fake = C.c_void_p(1 << 20)
    f = msqd.fdtd_fields(*([fake] * 11), fake)
    st = msqd.cpl_state(fake, fake, fake, fake, fake, fake, fake, fake, fake, fake, f, fake, fake)
    src = np.zeros(1)
    for every, code in [(5, msqd.MSQD_EINVAL), (-1, msqd.MSQD_EINVAL)]:
        d = msqd.cpl_desc(qd, fd, 8, 1.0, every)
        rc = msqd.lib.coupled_step(C.byref(d), C.byref(st), src.ctypes.data_as(C.POINTER(C.c_double)),
                                   0, 1, None)
        assert rc == code, (every, rc, msqd.last_error())
    assert "mol_every" in msqd.last_error()
    d = msqd.cpl_desc(qd, fd, 8, 1.0, 5)
    rc = msqd.lib.coupled_step(C.byref(d), C.byref(st), src.ctypes.data_as(C.POINTER(C.c_double)),
                               0, 1, None)
    assert "mol_every" in msqd.last_error() and rc == msqd.MSQD_EINVAL


def test_bloch_validation(msqd):
    d = msqd.bloch_desc(10, msqd.FP64, 0.3, 1.0, 0.0, 0.0, -0.1)
    assert msqd.lib.bloch_step(C.byref(d), None, None, None, 1, None) == msqd.MSQD_EINVAL
    assert "dt_au" in msqd.last_error()
    d = msqd.bloch_desc(10, 9, 0.3, 1.0, 0.0, 0.0, 0.1)
    assert msqd.lib.bloch_init(C.byref(d), None, None) == msqd.MSQD_EPREC
    d = msqd.bloch_desc(10, msqd.FP64, 0.3, 1.0, -1.0, 0.0, 0.1)
    assert msqd.lib.bloch_step(C.byref(d), None, None, None, 1, None) == msqd.MSQD_EINVAL
    d = msqd.bloch_desc(10, msqd.FP64, 0.3, 1.0, 0.0, 0.0, 0.1)
    assert msqd.lib.bloch_step(C.byref(d), None, None, None, 1, None) == msqd.MSQD_EINVAL
    assert "NULL" in msqd.last_error()


def test_jm_basis_validation(msqd):
    """The (j, m) basis is provided for 1 <= j_max <= 5, within one
    workgroup's threads and LDS; its workspace carries the coupling tables
    for j_max >= 2; an unknown basis value is rejected before anything
    touches a device."""
    def ws(n_r, j_max, prec=msqd.FP64):
        d = msqd.qd_desc(4, n_r, j_max, prec, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, msqd.BASIS_JM)
        return msqd.lib.qd_workspace_bytes(C.byref(d))

    assert ws(128, 1) > 0
    base = {jm: ws(128, jm, msqd.FP32) for jm in range(1, 6)}
    # the general tables: sum (2j+1)^2 + sum (j_max+1-a)^2 + (j_max+1)(j_max+2)/2 + 3 (j_max+1)^2
    # doubles after the common tables, then (256-aligned) the partial sums of
    # dipole_readout: one block of 1024 molecules x (3 dipole components,
    # norm, yield) here, against (1, norm, yield) in the m = 0 basis
    for jm in range(2, 6):
        n = sum((2 * j + 1) ** 2 for j in range(jm + 1)) + sum((jm + 1 - a) ** 2 for a in range(jm + 1)) \
            + (jm + 1) * (jm + 2) // 2 + 3 * (jm + 1) ** 2
        d0 = msqd.qd_desc(4, 128, jm, msqd.FP32, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, msqd.BASIS_M0)
        common = msqd.lib.qd_workspace_bytes(C.byref(d0)) - 8 * 3
        assert common % 256 == 0
        assert base[jm] == (common + 8 * n + 255) // 256 * 256 + 8 * 5
    assert ws(256, 5, msqd.MIXED) > 0
    for n_r, jm, prec in [(128, 0, msqd.FP64), (128, 6, msqd.FP32)]:
        assert ws(n_r, jm, prec) == 0
        assert "1 <= j_max <= 5" in msqd.last_error()
    # complex128 at n_r = 256 (16 lanes x 72 lines) and complex64 at n_r = 512
    # (16 lanes x 72 lines) exceed one workgroup; complex128 at n_r = 256 with
    # j_max = 4 exceeds its LDS
    for n_r, jm, prec in [(256, 5, msqd.FP64), (512, 5, msqd.FP32), (256, 4, msqd.FP64)]:
        assert ws(n_r, jm, prec) == 0
        assert "too large for one workgroup" in msqd.last_error()
    assert ws(512, 4, msqd.FP32) > 0 and ws(512, 2, msqd.FP64) > 0 and ws(256, 3, msqd.FP64) > 0
    d = msqd.qd_desc(4, 128, 1, msqd.FP64, 1.0, 12.0, 1e4, 0.1379, 2.0, 8.0, 7)
    assert msqd.lib.qd_workspace_bytes(C.byref(d)) == 0


def test_map_planes_and_held_plane_validation(msqd):
    """map_planes gives the z range of the occupied cells; coupled_step rejects
    a held-current array whose planes leave the grid, before any launch (the
    device pointers are placeholders, never touched)."""
    nx, ny, nz = 8, 6, 10
    plane = nx * ny
    assert msqd.map_planes(np.array([3 * plane + 5, 3 * plane + 7, 6 * plane]), nx, ny, nz) == (3, 4)
    assert msqd.map_planes(np.array([0]), nx, ny, nz) == (0, 1)
    assert msqd.map_planes(np.array([nz * plane - 1]), nx, ny, nz) == (nz - 1, 1)
    for bad in [np.array([nz * plane]), np.array([-1]), np.array([], np.int32)]:
        with pytest.raises(msqd.MsqdError):
            msqd.map_planes(bad, nx, ny, nz)
    from workloads import get_config
    cfg = get_config("cfg0")
    qd = msqd.qd_desc(64, cfg.n_r, cfg.j_max, msqd.FP64, cfg.r_min, cfg.r_max, cfg.mass,
                      cfg.dt_au, cfg.absorb_width, cfg.r_diss)
    fd = msqd.fdtd_desc_from_config(cfg, "fp64")
    fake = C.c_void_p(1 << 20)
    f = msqd.fdtd_fields(*([fake] * 11), fake)
    st = msqd.cpl_state(fake, fake, fake, fake, fake, fake, fake, fake, fake, fake, f, fake, fake)
    st.E_held = fake
    src = np.zeros(1)
    for k0, nk in [(0, 0), (-1, 2), (cfg.nz - 1, 2)]:
        d = msqd.cpl_desc(qd, fd, 8, 1.0, 1, k0, nk)
        rc = msqd.lib.coupled_step(C.byref(d), C.byref(st), src.ctypes.data_as(C.POINTER(C.c_double)),
                                   0, 1, None)
        assert rc == msqd.MSQD_EINVAL and "held planes" in msqd.last_error(), (k0, nk, rc)
    st.E_held = C.c_void_p((1 << 20) + 8)
    d = msqd.cpl_desc(qd, fd, 8, 1.0, 1, 10, 4)
    rc = msqd.lib.coupled_step(C.byref(d), C.byref(st), src.ctypes.data_as(C.POINTER(C.c_double)), 0, 1, None)
    assert rc == msqd.MSQD_EINVAL and "E_held misaligned" in msqd.last_error()
