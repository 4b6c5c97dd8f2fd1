/*
 * msqd.h - C ABI of the MI355X library for the coupled Maxwell-Schroedinger
 * step of Sukharev, "Efficient parallel strategy for molecular plasmonics"
 * (arXiv 2209.04487).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers are caller-owned (PyTorch allocations), contiguous and
 *    at least 16-byte aligned.  The library never allocates or frees device
 *    memory.  Host pointers are read during the call only.
 *  - `stream` is a hipStream_t passed as void*.  Calls only enqueue work on it
 *    (init calls also wait for their own host-to-device table copies); results
 *    land in device buffers.
 *  - Return value: MSQD_OK (0) or a negative MSQD_E* code.  On a negative
 *    return nothing was launched; msqd_last_error() gives a thread-local
 *    message.
 *  - Units: the molecule side is in Hartree atomic units, the field side in
 *    SI (the paper gives its potential parameters in a.u. and writes Maxwell's
 *    equations in SI).  Conversions use CODATA 2018 values.
 *  - Precision `prec`: MSQD_FP64 (complex128 wavepackets, float64 fields),
 *    MSQD_FP32 (complex64 wavepackets and FP32 J<->angle transform, float32
 *    fields), MSQD_MIXED (complex64 wavepackets, the J<->angle transform on
 *    BF16 matrix cores with a hi/lo split and FP32 accumulation, float32
 *    fields).  Per-molecule and per-cell reductions (absorbed norm, dipole,
 *    norm, yield, cell polarisation) are float64 in every form.
 *
 * Wavepacket layout: psi[mol][s][J][r] complex (interleaved re, im), s = 0
 * ground, 1 excited, J = 0..j_max (m = 0), r = 0..n_r-1 on the periodic grid
 * r_k = r_min + k (r_max - r_min)/n_r.
 * Field layout: every component is [nz][ny][nx] with x fastest; E_x sits at
 * (i+1/2, j, k), E_y (i, j+1/2, k), E_z (i, j, k+1/2), H_x (i, j+1/2, k+1/2),
 * H_y (i+1/2, j, k+1/2), H_z (i+1/2, j+1/2, k) in cell units.
 */
#ifndef MSQD_H
#define MSQD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MSQD_OK = 0,
  MSQD_EINVAL = -1,     /* null pointer, bad extent or alignment            */
  MSQD_ESHAPE = -2,     /* sizes inconsistent with each other / workspace   */
  MSQD_EPREC = -3,      /* unknown precision                                */
  MSQD_EUNSUP = -4,     /* unsupported size (n_r not 2^k in [64,512], ...)  */
  MSQD_EDEVICE = -5,    /* HIP runtime error                                */
  MSQD_ENONFINITE = -6  /* a readout found NaN/Inf                          */
};

enum { MSQD_FP64 = 0, MSQD_FP32 = 1, MSQD_MIXED = 2 };
/* rotational basis of the wavepackets (qd_desc.basis): m = 0 J lines, or
 * the full (j, m) basis with all three field components (Eq. (3)) */
enum { MSQD_BASIS_M0 = 0, MSQD_BASIS_JM = 1 };

/* Thread-local message of the last failing call ("" if none). */
const char* msqd_last_error(void);
/* Library version (major*10000 + minor*100 + patch). */
int msqd_version(void);

/* Instrumentation of the molecular step inside coupled_step (host only, per
 * calling thread; not needed for any computation).  msqd_mol_timing_begin
 * creates max_launches pairs of HIP timing events (1 <= max_launches <=
 * 2^20); until msqd_mol_timing_end, every coupled_step call on this thread
 * records one pair around each of its molecular-step launches, on the
 * call's stream, for the first max_launches launches.
 * msqd_mol_timing_end waits for the recorded events, writes the summed
 * duration of the recorded launches (ms) and their number, and destroys the
 * events.  Errors: MSQD_EINVAL (bad count, NULL output, end without begin),
 * MSQD_EDEVICE (event creation or query failed). */
int msqd_mol_timing_begin(int32_t max_launches);
int msqd_mol_timing_end(double* total_ms, int32_t* n_launches);

/* ------------------------------------------------------------------------
 * Molecules: two-state ro-vibrational wavepackets, Eqs. (3)-(5).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_mol;          /* molecules in the batch                        */
  int32_t n_r;            /* radial points: 64, 128, 256 or 512            */
  int32_t j_max;          /* rotational basis J = 0..j_max (m = 0), <= 15  */
  int32_t prec;           /* MSQD_FP64 | MSQD_FP32 | MSQD_MIXED            */
  double r_min, r_max;    /* periodic radial box, bohr (r_max excluded)    */
  double mass_au;         /* reduced mass, electron masses                 */
  double dt_au;           /* molecular time step, atomic units             */
  double absorb_width_au; /* cos^(1/8) absorber over [r_max - w, r_max); 0 = none */
  double r_diss_au;       /* dissociated population counts r > r_diss      */
  int32_t basis;          /* MSQD_BASIS_M0: J lines with m = 0, the field
                             along the quantisation axis (E_mol, d_mol: one
                             value per molecule); MSQD_BASIS_JM: all
                             (j, m) with j <= j_max, 1 <= j_max <= 5, all
                             three field components (E_mol, d_mol:
                             [n_mol][3] = x, y, z), psi lines ordered
                             b = j^2 + m + j.  One workgroup holds a
                             molecule: 2 (j_max+1)^2 lines of n_r/R1 lanes
                             (R1 = 32 for complex64 at n_r >= 256, 16 for
                             complex128 at n_r = 256 and for n_r = 128, 8 at
                             n_r = 64) must stay within 1024 threads and
                             160 KB of LDS, else MSQD_EUNSUP (e.g. complex128
                             at n_r = 256 takes j_max <= 3).  This basis has
                             no J<->angle contraction: MSQD_FP32 and
                             MSQD_MIXED run the same complex64 kernel.       */
} qd_desc;

/* Bytes of device workspace (tables, a status word, and the partial sums of
 * dipole_readout's ensemble sums: 8 (nc + 2) ceil(n_mol / 1024) bytes, nc =
 * 1 or 3 dipole components) for qd_* calls; 0 (with the message) for an
 * invalid or unsupported descriptor.  With basis = MSQD_BASIS_JM and
 * j_max >= 2 it includes the tables of the general coupling (the
 * Wigner-rotation eigenvectors of J_x, the per-m' eigen-decompositions of
 * cos(theta) and the dipole matrix elements).  qd_init rejects a smaller
 * ws_bytes with MSQD_ESHAPE. */
size_t qd_workspace_bytes(const qd_desc* d);

/* Build the split-operator tables (Eq. (5) phases on the grid, the
 * Gauss-Legendre angular grid that integrates the angular part of Eq. (4)
 * exactly on the truncated basis, absorber mask) into `ws` and set every
 * molecule to (g, J=0) with radial function psi0 (host [n_r], real),
 * all other channels 0; absorbed[] := 0.
 * U_g, U_e: host [n_r] surfaces (hartree); mu12: host [n_r] transition
 * dipole (e a0), all sampled on the grid. */
int qd_init(const qd_desc* d, const double* U_g, const double* U_e, const double* mu12,
            const double* psi0, void* ws, size_t ws_bytes, void* psi, double* absorbed,
            void* stream);

/* Host only (no device, no stream): the tables of the general (j, m)
 * coupling (2 <= j_max <= 5) that qd_init places in the workspace, as
 * doubles, for inspection and host-side checks.  Layout, in order:
 *   O^(j), j = 0..j_max: eigenvectors of J_x on the block j, (2j+1)^2 each,
 *     row m + j, column k for the eigenvalue k - j (the Wigner matrices
 *     follow as d^j_{m m'}(beta) = sum_k O_{mk} O_{m'k} cos(pi/2 (m'-m) - beta (k-j)));
 *   Q^(a), a = |m'| = 0..j_max: eigenvectors of cos(theta) on the states
 *     j = a..j_max of one m', (j_max+1-a)^2 each, row j - a, column k;
 *   x^(a): the matching eigenvalues, ascending, j_max+1-a each;
 *   per basis state b = j^2 + m + j: <j+1,m|cos th|j,m>,
 *     <j+1,m+1|sin th e^{i ph}|j,m>, <j-1,m+1|sin th e^{i ph}|j,m> (0 where
 *     the target state lies outside the basis).
 * qd_jm_tables_size: the number of doubles (0 if j_max is outside 2..5).
 * Errors: MSQD_EUNSUP (j_max), MSQD_EINVAL (NULL), MSQD_ESHAPE (n_out too
 * small), MSQD_EDEVICE (an eigen-decomposition failed to converge; not
 * expected for these sizes). */
size_t qd_jm_tables_size(int32_t j_max);
int qd_jm_tables(int32_t j_max, double* out, size_t n_out);

/* Advance every molecule n_steps split-operator steps (K/2 V/2 C(E) V/2 K/2,
 * then the absorber) under a field held constant over the call.
 * E_mol: device [n_mol] float64 field along the quantisation axis (au).
 * absorbed: device [n_mol] float64, accumulated.  d_mol: device [n_mol]
 * float64 dipole <mu12 cos(theta) sigma_x> (e a0) after the last step, or
 * NULL.
 * With basis = MSQD_BASIS_JM: E_mol is [n_mol][3] (E_x, E_y, E_z) and d_mol
 * [n_mol][3], the dipole <mu12 d_c sigma_x> along x, y, z; the coupling is
 * exp(i mu12 dt sigma_x (x) sum_c E_c D_c), exact on the truncated basis,
 * D_c the direction cosines of the molecular axis (Eq. (3) with all m):
 * a closed form for j_max = 1; for j_max >= 2 the rotation of the field
 * direction onto z, per-m' Gauss transforms of cos(theta), the 2x2 rotation
 * of each eigenvector's (g, e) pair and the way back. */
int qd_step(const qd_desc* d, const void* ws, void* psi, const double* E_mol,
            double* absorbed, double* d_mol, int32_t n_steps, void* stream);

/* Per-molecule readouts of the current state (float64, device) and their
 * ensemble sums.  The dipole is the expectation of mu12(r) cos(theta)
 * sigma_x, the quantity whose density is the mean-field polarisation that
 * returns to Ampere's law (section on the coupled equations, Eqs. (1), (4));
 * the yield is the dissociated population (norm beyond r_diss plus the
 * absorbed norm) of the section on collective dissociation dynamics.
 *   d_mol     [n_mol] (e a0), or [n_mol][3] in the (j, m) basis;
 *   norm_mol  [n_mol] sum |psi|^2 dr;
 *   yield_mol [n_mol] norm beyond r_diss plus absorbed;
 *   sums      [nc + 2] FP64 = (sum d (nc = 1, or the x, y, z sums: nc = 3),
 *             sum norm, sum yield) over all molecules, in a fixed two-stage
 *             order (blocks of 1024 consecutive molecules, then the block
 *             partials), bit-reproducible for a given n_mol; or NULL.  The
 *             stage-one partials use the tail of ws (qd_workspace_bytes).
 * Per-molecule outputs may be NULL when sums is NULL; sums needs all three
 * (it reduces them): MSQD_EINVAL otherwise.  With n_mol = 0 only sums is
 * written (zeros).  The state is not modified. */
int dipole_readout(const qd_desc* d, const void* ws, const void* psi, const double* absorbed,
                   double* d_mol, double* norm_mol, double* yield_mol, double* sums, void* stream);

/* dipole_readout for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, results and errors, but the stage-one partial sums of
 * `sums` go to a static device array of the library (40 KB per GPU, held
 * until the process ends) instead of the tail of ws, so ws only needs the
 * tables (qd_workspace_bytes still covers it).  It calls no hipMalloc,
 * hipFree or allocating routine.  Limit: with sums, n_mol <= 1,048,576
 * (1024 blocks of 1024 molecules), else MSQD_EUNSUP and nothing is launched.
 * Every call on one GPU shares that GPU's array, so calls whose sums overlap
 * in time on one GPU (different streams, or threads) race; calls ordered on
 * one stream do not.  The first call on a device looks up the array's
 * device address (hipGetSymbolAddress) with that device current. */
int dipole_readout_noalloc(const qd_desc* d, const void* ws, const void* psi, const double* absorbed,
                           double* d_mol, double* norm_mol, double* yield_mol, double* sums, void* stream);

/* Excited-state internuclear distance, Eq. (8): per molecule (float64,
 * device) r_num = <chi_e|R|chi_e> = sum_{J,k} r_k |psi_e,J(r_k)|^2 dr and
 * pop = <chi_e|chi_e>; the ratio is the molecule's <R>_e.  sums: device
 * float64 [3] = (sum r_num, sum pop, their ratio: the ensemble <R>_e, each
 * molecule weighted by its excited population; NaN while that population is
 * exactly zero) over all molecules in a fixed order, or NULL.  With
 * n_mol = 0 nothing is written.  ws is unused but validated like the other
 * readouts.  Errors: MSQD_EINVAL for NULL outputs. */
int excited_r_readout(const qd_desc* d, const void* ws, const void* psi, double* r_num, double* pop,
                      double* sums, void* stream);

/* Synchronise `stream`, then report MSQD_ENONFINITE (and clear the flag) if
 * any molecular step since the last check produced a non-finite dipole,
 * norm or absorbed norm; MSQD_OK otherwise.  ws is a qd workspace. */
int msqd_check_status(const void* ws, void* stream);

/* ------------------------------------------------------------------------
 * Fields: Yee leap-frog of Eq. (1) with the Drude current of Eq. (2).
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;     /* cells; x and y periodic; nz <= 65535, nx*ny*nz <= 2e9 (else MSQD_EUNSUP) */
  int32_t npml;           /* CPML thickness (cells) at each z end, >= 1     */
  int32_t prec;           /* MSQD_FP64 | MSQD_FP32 | MSQD_MIXED (FP32 fields) */
  int32_t metal_id;       /* material id that carries the Drude current     */
  double dx;              /* cell size (m)                                  */
  double dt;              /* time step (s)                                  */
  double eps_r[4];        /* relative permittivity per material id (eps_inf for the metal) */
  double drude_wp;        /* plasma frequency (rad/s), Eq. (2)              */
  double drude_gamma;     /* damping (rad/s), Eq. (2)                       */
  double cpml_m;          /* polynomial grading order                       */
  double sigma_max_lo, sigma_max_hi;  /* CPML sigma_max at the low / high z end (S/m) */
  double kappa_max, alpha_max;        /* CPML kappa_max (>= 1), alpha_max (S/m) */
  int32_t src_k;          /* plane of the soft current sheet on E_x         */
  int32_t mon_k;          /* detection plane (npml < mon_k < nz - npml)     */
  int32_t n_freq;         /* monitor frequencies (0 = no monitor, at most 65536) */
  int32_t mon_every;      /* monitor sampling interval in steps             */
  int32_t mon_k2;         /* second detection plane on the incident side for
                             reflection/absorption spectra (0 = none)       */
} fdtd_desc;

/* Device buffers of the field solver; element type is double (FP64) or
 * float (FP32/MIXED) for the field arrays. */
typedef struct {
  void *Ex, *Ey, *Ez, *Hx, *Hy, *Hz;   /* [nz][ny][nx] each                 */
  void *JDx, *JDy, *JDz;               /* Drude currents, [nz][ny][nx] each */
  void* psi;       /* CPML auxiliaries: 4 x [2*npml][ny][nx] (psi_Ex, psi_Ey, psi_Hx, psi_Hy),
                      planes k < npml then k >= nz - npml                    */
  uint8_t* mat;    /* [3][nz][ny][nx] material id per E-component location  */
  double* dft;     /* [planes][4][n_freq][ny][nx] complex128 (E_x, E_y, H_x,
                      H_y), planes = 2 with mon_k2, else 1; then the monitor's
                      staging area, [planes][8][4][ny][nx] float64, whose
                      contents between calls carry nothing (each call folds
                      its staged samples in before it returns); or NULL     */
} fdtd_fields;

size_t fdtd_workspace_bytes(const fdtd_desc* d);
/* Bytes of the CPML auxiliary buffer `psi` and of the monitor buffer `dft`
 * (accumulators and staging area; 0 without a monitor). */
size_t fdtd_psi_bytes(const fdtd_desc* d);
size_t fdtd_dft_bytes(const fdtd_desc* d);

/* Zero every field, copy the host material map mat_host [3][nz][ny][nx] to
 * f->mat, and build the CPML coefficient profiles and monitor frequencies
 * (host [n_freq], rad/s) into ws. */
int fdtd_init(const fdtd_desc* d, const uint8_t* mat_host, const double* freqs,
              const fdtd_fields* f, void* ws, size_t ws_bytes, void* stream);

/* One field step n -> n+1 without molecules: H^{n+1/2}, then E^{n+1} with the
 * Drude current and the source sheet J_x = -2 src_value/(eta0 dx) on plane
 * src_k (src_value = E_inc(t_{n+1/2}) in V/m), then a monitor sample when
 * (n+1) % mon_every == 0. */
int fdtd_step(const fdtd_desc* d, const fdtd_fields* f, const void* ws, int64_t n,
              double src_value, void* stream);

/* Plane-averaged z-flux S(w_f) = <1/2 Re(E_x H_y* - E_y H_x*)> of the monitor
 * DFTs into flux (device float64 [planes][n_freq]: the mon_k plane, then the
 * mon_k2 plane when set).  With a vacuum reference run's incident-side flux
 * S_ref: T = S(mon_k)/S_ref, R = 1 - S(mon_k2)/S_ref, A = 1 - T - R (the
 * short-pulse spectra of the section on 3D domain decomposition, Fig. 6a). */
int flux_readout(const fdtd_desc* d, const fdtd_fields* f, double* flux, void* stream);

/* Transmission, reflection and absorption spectra of the short-pulse runs
 * (section on 3D domain decomposition, Fig. 6a), per monitor frequency:
 *   T = S_trans / S_ref,  R = (S_ref - S_inc) / S_ref,  A = (S_inc - S_trans) / S_ref = 1 - T - R,
 * with flux the device float64 [2][n_freq] readout of a run with both
 * detection planes (S_trans on mon_k beyond the structure, S_inc on mon_k2
 * on the incident side, where the net flux is the incident minus the
 * reflected one) and flux_ref a device float64 [n_freq] incident-side flux of
 * a reference run without the structure.  tra: device float64 [3][n_freq] =
 * T, R, A.  Errors: MSQD_EINVAL for NULL pointers, no monitor, or no
 * second plane (d->mon_k2 = 0). */
int spectra_readout(const fdtd_desc* d, const double* flux, const double* flux_ref, double* tra, void* stream);

/* ------------------------------------------------------------------------
 * Coupling: molecules <-> cells, the self-consistent step.
 * ---------------------------------------------------------------------- */

/* Host helper: molecule -> flat E_x index and the CSR of occupied cells.
 * Molecules are placed with SplitMix64(seed), three words per molecule,
 * i = ((u>>11)*nx)>>53, j likewise, k = slab_k0 + ((u>>11)*slab_nk)>>53.
 * Outputs (host): cell_of_mol [n_mol], occ_cell [n_mol] (first *n_occ
 * used, increasing), occ_ptr [n_mol+1] (first *n_occ+1 used), mol_perm
 * [n_mol] (molecules cell by cell, increasing index inside a cell). */
int map_build(int32_t n_mol, int32_t nx, int32_t ny, int32_t nz, uint64_t seed,
              int32_t slab_k0, int32_t slab_nk, int32_t* cell_of_mol, int32_t* occ_cell,
              int32_t* occ_ptr, int32_t* mol_perm, int32_t* n_occ);

/* The same CSR for a caller-given cell_of_mol (host). */
int map_csr(int32_t n_mol, int32_t n_cells, const int32_t* cell_of_mol, int32_t* occ_cell,
            int32_t* occ_ptr, int32_t* mol_perm, int32_t* n_occ);

/* Host helper: the planes held_k0 .. held_k0 + held_nk - 1 that hold every
 * occupied cell (occ_cell: host [n_occ] flat E_x indices of an nx x ny x nz
 * grid), for cpl_desc's held-current array.  MSQD_EINVAL for n_occ < 1, a
 * NULL pointer or an index outside the grid. */
int map_planes(int32_t n_occ, const int32_t* occ_cell, int32_t nx, int32_t ny, int32_t nz,
               int32_t* held_k0, int32_t* held_nk);

typedef struct {
  qd_desc qd;
  fdtd_desc fd;
  int32_t n_occ;        /* occupied cells                                  */
  double mol_weight;    /* molecules represented by each simulated one     */
  int32_t mol_every;    /* M: molecules step every M field steps (0 or 1:
                           every step); qd.dt_au must equal M fd.dt in
                           atomic units (relative 1e-9)                     */
  int32_t held_k0;      /* with s->E_held: planes held_k0 .. held_k0 +      */
  int32_t held_nk;      /* held_nk - 1 hold every occupied cell (ignored
                           when s->E_held is NULL)                          */
} cpl_desc;

typedef struct {
  void* psi;                 /* wavepackets (see qd_step)                  */
  double* absorbed;          /* [n_mol]                                    */
  double* d_mol;             /* [n_mol] dipoles after the last step        */
  double* E_mol;             /* [n_mol] field seen in the last step (au)   */
  double* P_c;               /* [n_occ] cell polarisation (C/m^2)          */
  double* J_mol;             /* [n_occ] last polarisation current (A/m^2)  */
  const int32_t* cell_of_mol;  /* [n_mol] flat E_x index                   */
  const int32_t* occ_cell;     /* [n_occ]                                  */
  const int32_t* occ_ptr;      /* [n_occ+1]                                */
  const int32_t* mol_perm;     /* [n_mol]                                  */
  fdtd_fields f;
  const void* qd_ws;
  const void* fd_ws;
  void* psi_next;            /* NULL: the molecular step updates psi in
                                place.  Else (m = 0 basis, n_steps = 1) it
                                reads psi and writes the stepped wavepackets
                                to psi_next (same layout, caller-owned, 16-byte
                                aligned, not overlapping psi), leaving psi as
                                it was, so that a gradient's segment recompute
                                keeps every step's state without copies.  With
                                mol_every > 1 only the steps where the
                                molecules step (n % mol_every == 0) write it. */
  void* E_held;              /* NULL: the molecular current is subtracted from
                                E by a pass after each E update.  Else the
                                E update subtracts it itself, reading this
                                array: [ncomp][held_nk][ny][nx] in the field
                                precision (ncomp = 3 in the (j, m) basis,
                                else 1), caller-owned, 16-byte aligned,
                                zero-filled by the caller before its first
                                use and again whenever the occupied cells
                                change.  The library keeps the molecular
                                term in it at each occupied edge (FP32 fields:
                                dt/(eps0 eps_r) J_mol rounded to float; FP64:
                                J_mol, the E update fusing the product into
                                its subtraction); a call
                                that starts between molecular updates
                                rebuilds it from J_mol, so J_mol and P_c
                                alone carry the state (checkpoints need not
                                hold it).  An occupied cell outside the held
                                planes sets its E components to NaN. */
} cpl_state;

/* n_steps coupled steps from step n0 (section on molecular mapping, with
 * Eqs. (1), (2), (4), (5)): H^{n+1/2}; E_mol = E_x^n at each molecule's edge;
 * every molecule one step under E_mol; d_i; P_c^{n+1} = (w/dx^3) sum_{i in c}
 * d_i (e a0) in CSR order and J_mol = (P_c^{n+1} - P_c^n)/dt; E^{n+1} with
 * Drude, molecular and source currents; monitor sample.
 * Multi-rate (d->mol_every = M > 1, the paper's molecules-every-40th-step
 * scheme): the molecular part runs only at steps with n % M == 0, each
 * molecule taking one step of M dt under E_x^n; J_mol = (P_new - P_old)/(M dt)
 * is then applied unchanged at every field step until the next update.
 * src_values: host [n_steps], E_inc(t_{n+1/2}) in V/m.
 * With s->E_held set the results are bit-identical to those without it: the
 * new J_mol is formed after the molecular step and before the E update, which
 * then subtracts it, so the steps between updates launch no separate pass.
 * Errors: MSQD_EINVAL for a step/precision mismatch (qd.dt_au != M fd.dt),
 * for s->E_held misaligned or with held planes outside the grid,
 * and for s->psi_next set with n_steps != 1, misaligned or equal to s->psi;
 * MSQD_EUNSUP for s->psi_next set in the (j, m) basis. */
int coupled_step(const cpl_desc* d, const cpl_state* s, const double* src_values, int64_t n0,
                 int32_t n_steps, void* stream);

/* ------------------------------------------------------------------------
 * Frozen two-level (Bloch) emitters: the paper's comparison workload in the
 * section on molecular mapping, where the ro-vibrational degrees of freedom
 * are frozen and each molecule obeys the Bloch equations, integrated by the
 * classical fourth-order Runge-Kutta scheme.  Atomic units; interaction
 * -mu E sigma_x with the field along the dipole, V = -mu E:
 *   d rho_ee/dt = 2 V Im(rho_ge) - gamma1 rho_ee
 *   d rho_ge/dt = (i omega0 - gamma2) rho_ge - i V (2 rho_ee - 1)
 * The field is held over each step.  The emitter's dipole is
 * d = 2 mu Re(rho_ge).
 * State: caller-owned device planes [3][n] = (rho_ee, Re rho_ge, Im rho_ge),
 * double for MSQD_FP64, float for MSQD_FP32 and MSQD_MIXED, 16-byte aligned.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n;            /* emitters (>= 0)                                  */
  int32_t prec;         /* MSQD_FP64 | MSQD_FP32 | MSQD_MIXED (= FP32 here)  */
  double omega0_au;     /* transition frequency                             */
  double mu_au;         /* transition dipole along the field                */
  double gamma1_au;     /* population decay rate (>= 0)                     */
  double gamma2_au;     /* coherence decay rate (>= 0)                      */
  double dt_au;         /* step (> 0)                                       */
} bloch_desc;

/* state := the ground state (rho_ee = rho_ge = 0).  Errors: MSQD_EINVAL. */
int bloch_init(const bloch_desc* d, void* state, void* stream);

/* n_steps RK4 steps under E (device double [n], au) held over the steps;
 * d_out: device double [n] dipoles after the steps (au), or NULL.
 * n_steps = 0 only writes d_out.  Errors: MSQD_EINVAL, MSQD_EPREC. */
int bloch_step(const bloch_desc* d, void* state, const double* E, double* d_out, int32_t n_steps,
               void* stream);

/* The coupled step with Bloch emitters in place of the wavepackets: the same
 * H update, gather of E_x^n at each emitter's edge, per-cell polarisation in
 * CSR order, polarisation current and E update as coupled_step (M = 1).
 * bl.dt_au must equal fd.dt in atomic units (relative 1e-9); bl.prec and
 * fd.prec are both FP64 or both reduced. */
typedef struct {
  bloch_desc bl;
  fdtd_desc fd;
  int32_t n_occ;
  double weight;        /* emitters represented by each simulated one       */
} cpl_bloch_desc;

typedef struct {
  void* state;                 /* [3][n] (see bloch_step)                   */
  double* d_mol;               /* [n] dipoles after the last step           */
  double* E_mol;               /* [n] field seen in the last step (au)      */
  double* P_c;                 /* [n_occ]                                   */
  double* J_mol;               /* [n_occ]                                   */
  const int32_t* cell_of_mol;  /* [n]                                       */
  const int32_t* occ_cell;     /* [n_occ]                                   */
  const int32_t* occ_ptr;      /* [n_occ+1]                                 */
  const int32_t* mol_perm;     /* [n]                                       */
  fdtd_fields f;
  const void* fd_ws;
} cpl_bloch_state;

int coupled_bloch_step(const cpl_bloch_desc* d, const cpl_bloch_state* s, const double* src_values,
                       int64_t n0, int32_t n_steps, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint of the coupled step (reverse mode), for gradients of the
 * dissociated population Y = mean_i [sum_{r > r_diss} |psi_i|^2 dr +
 * absorbed_i] with respect to the incident-field samples.
 * For complex psi the adjoint is dY/dRe(psi) + i dY/dIm(psi).
 * Supported in the MSQD_FP64 and MSQD_FP32 forms, for any mol_every (with
 * mol_every > 1 the molecules step only at n % mol_every == 0, and the held
 * current's adjoint lJ carries the field sensitivity of the held steps back
 * to the update that set the current).
 * ---------------------------------------------------------------------- */
typedef struct {
  void* lpsi;        /* adjoint of psi, same layout and type              */
  double* labs;      /* [n_mol] adjoint of the absorbed norms             */
  double* lP;        /* [n_occ] adjoint of the cell polarisation          */
  double* ld;        /* [n_mol] scratch: adjoint of the step's dipoles    */
  double* lE;        /* [n_mol] scratch: adjoint of the gathered fields   */
  fdtd_fields lf;    /* adjoint fields (E, H, J_D, CPML psi); mat, dft unused */
  void* scratch;     /* adjoint_scratch_bytes() of device memory          */
  double* lJ;        /* [n_occ] adjoint of the held molecular current;
                        needed with mol_every > 1 (zeroed by
                        adjoint_init_yield), ignored otherwise (may be NULL) */
} cpl_adj;

size_t adjoint_scratch_bytes(const cpl_desc* d);

/* Set the adjoint to dY/d(state) at the end of a run: lpsi = (2 dr/n_mol) psi
 * for r > r_diss, labs = 1/n_mol, everything else 0.  s->psi is the final
 * wavepacket. */
int adjoint_init_yield(const cpl_desc* d, const cpl_state* s, cpl_adj* adj, void* stream);

/* One reverse step n: with adj holding dY/d(state after step n), overwrite
 * it with dY/d(state before step n) and write g_src[0] = dY/dsrc_value[n]
 * (device float64).  psi_n and E_mol_n are the wavepackets before step n
 * and the field it gathered (recorded by a forward recompute; with
 * mol_every > 1 they are read only at the update steps n % mol_every == 0);
 * psi_np1 is the wavepackets after step n (the recompute's next state, e.g.
 * written there by coupled_step's psi_next), or NULL: given, the molecular
 * adjoint reads the absorber's input back from it instead of recomputing
 * the second half of the forward step.  In the FP64 form the step then also
 * uses psi_np1 as its scratch (it holds the coupling's input there), so its
 * contents are undefined on return: a reverse sweep passes each recorded
 * state as psi_np1 only after its last use as psi_n.  s supplies the maps,
 * tables and material map of the forward system.
 * Errors: MSQD_EINVAL also for n < 0 and for psi_np1 misaligned or equal
 * to psi_n. */
int adjoint_step(const cpl_desc* d, const cpl_state* s, const void* psi_n, void* psi_np1,
                 const double* E_mol_n, cpl_adj* adj, int64_t n, double* g_src, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSQD_H */
