// C ABI of libmsqd: argument validation, workspace tables, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.h"
#include "bloch.h"
#include "readout.h"
#include "fdtd.h"
#include "host_tables.h"
#include "mol.h"
#include "mol_jmg.h"

namespace msqd {

static thread_local std::string g_err;

// Molecular-launch timing of the calling thread (msqd_mol_timing_begin/end):
// event pairs recorded around the molecular-step launches of coupled_step
struct MolTiming {
  std::vector<hipEvent_t> b, e;
  int n_rec = 0;
  bool armed = false;
};
static thread_local MolTiming g_timing;

static void timing_mark(bool before, hipStream_t s) {
  MolTiming& t = g_timing;
  if (!t.armed || t.n_rec >= static_cast<int>(t.b.size())) return;
  (void)hipEventRecord(before ? t.b[t.n_rec] : t.e[t.n_rec], s);
  if (!before) ++t.n_rec;
}

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int check_hip(hipError_t e, const char* what) {
  g_err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return MSQD_EDEVICE;
}

static inline size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

QdLayout qd_layout(int n_r, int nj) {
  QdLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t nr = n_r, J = nj;
  L.status = take(16);
  L.psi0 = take(8 * nr);
  L.kin_d = take(16 * nr);
  L.tw_d = take(16 * 32 * 32);
  L.vph_d = take(16 * 2 * J * nr);
  L.x_d = take(8 * J);
  L.mudt_d = take(8 * nr);
  L.mask_d = take(8 * nr);
  L.mu_d = take(8 * nr);
  L.cj_d = take(8 * J);
  L.kin_f = take(8 * nr);
  L.tw_f = take(8 * 32 * 32);
  L.tw_fs = take(8 * 32 * 32);
  L.vph_f = take(8 * 2 * J * nr);
  L.x_f = take(4 * J);
  L.mudt_f = take(4 * nr);
  L.mask_f = take(4 * nr);
  L.tmfrag = take(4 * 64 * 4 * 2);  // bf16 fragments: 4 operand blocks x 64 lanes x 4 values
  L.tmfrag_d = take(2 * 64 * 4 * 8);
  L.tmfrag_f = take(2 * 64 * 4 * 4);
  L.total = o;
  return L;
}

FdLayout fd_layout(const fdtd_desc* d) {
  FdLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t nz = d->nz;
  L.bE = take(8 * nz);
  L.aE = take(8 * nz);
  L.kE = take(8 * nz);
  L.bH = take(8 * nz);
  L.aH = take(8 * nz);
  L.kH = take(8 * nz);
  L.bEf = take(4 * nz);
  L.aEf = take(4 * nz);
  L.kEf = take(4 * nz);
  L.bHf = take(4 * nz);
  L.aHf = take(4 * nz);
  L.kHf = take(4 * nz);
  L.freqs = take(8 * static_cast<size_t>(d->n_freq > 0 ? d->n_freq : 1));
  L.total = o;
  return L;
}

size_t mol_lds_bytes(int n_r, int nj, int prec) {
  const size_t el = prec == MSQD_FP64 ? 16 : 8;
  const int r1 = fft_r1(n_r, static_cast<int>(el / 2));
  const int r2 = n_r / r1;
  // exchange rounds of the forward step (two for complex64 lines with an
  // even number of columns per lane)
  const int split = (el == 8 && (r1 / r2) % 2 == 0) ? 2 : 1;
  // tables staged in LDS: kinetic factors, twiddles, mask, and the
  // contraction operands (2 KB of matrix-core fragments, 16 angle nodes)
  const bool staged = el == 8;
  const size_t tables =
      staged ? (el * n_r + el * static_cast<size_t>(r1) * r1 + (el / 2) * n_r + 15) / 16 * 16 + 2048 + 64 : 0;
  // lines, the spare row of the contractions (one round of radial points),
  // the reduction scratch
  return tables + el * (static_cast<size_t>(lds_line_start(2 * nj, n_r / split + r2, static_cast<int>(el))) +
                        n_r / split) +
         16 * 4 * sizeof(double);
}

size_t mol_lds_limit() {
  static std::atomic<int> cached{-1};
  int v = cached.load(std::memory_order_acquire);
  if (v < 0) {
    int dev = 0;
    v = 0;
    if (!(hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0))
      v = 64 * 1024;
    (void)hipGetLastError();
    cached.store(v, std::memory_order_release);
  }
  return static_cast<size_t>(v);
}

hipError_t allow_large_lds(const void* kernel, std::atomic<unsigned long long>& done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const unsigned long long bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0ull;
  if (bit != 0 && (done.load(std::memory_order_acquire) & bit) != 0) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(mol_lds_limit()));
  (void)hipGetLastError();
  if (e == hipSuccess && bit != 0) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// ------------------------------------------------------------ validation
static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// wavepacket lines per molecule: 2 states x (J lines, or (j_max+1)^2 (j, m) lines)
static int qd_lines(const qd_desc* d) {
  const int nj = d->j_max + 1;
  return 2 * (d->basis == MSQD_BASIS_JM ? nj * nj : nj);
}

static int check_qd(const qd_desc* d) {
  if (!d) return fail(MSQD_EINVAL, "qd_desc is NULL");
  if (d->n_mol < 0) return fail(MSQD_EINVAL, "n_mol < 0");
  if (d->n_r != 64 && d->n_r != 128 && d->n_r != 256 && d->n_r != 512)
    return fail(MSQD_EUNSUP, "n_r must be 64, 128, 256 or 512");
  if (d->j_max < 0 || d->j_max + 1 > kMaxNJ) return fail(MSQD_EUNSUP, "j_max must be in [0, 15]");
  if (d->prec != MSQD_FP64 && d->prec != MSQD_FP32 && d->prec != MSQD_MIXED)
    return fail(MSQD_EPREC, "unknown precision");
  if (!(d->r_max > d->r_min) || !(d->r_min > 0.0)) return fail(MSQD_EINVAL, "need 0 < r_min < r_max");
  if (d->basis != MSQD_BASIS_M0 && d->basis != MSQD_BASIS_JM) return fail(MSQD_EINVAL, "unknown basis");
  if (d->basis == MSQD_BASIS_JM) {
    if (d->j_max < 1 || d->j_max > kJmgMax)
      return fail(MSQD_EUNSUP, "the (j, m) basis is provided for 1 <= j_max <= " + std::to_string(kJmgMax));
    size_t lds = 0;
    if (d->j_max >= 2 && !jmg_supported(d->n_r, d->prec != MSQD_FP64, d->j_max, &lds))
      return fail(MSQD_EUNSUP, "(j, m) basis: n_r x (j_max+1)^2 too large for one workgroup in this precision (" +
                                   std::to_string(lds) + " bytes of LDS, " +
                                   std::to_string(qd_lines(d) * (d->n_r / fft_r1(d->n_r, d->prec == MSQD_FP64 ? 8 : 4))) +
                                   " threads)");
  }
  if (!(d->mass_au > 0.0) || !(d->dt_au > 0.0)) return fail(MSQD_EINVAL, "mass and dt must be > 0");
  if (d->absorb_width_au < 0.0 || d->absorb_width_au > d->r_max - d->r_min)
    return fail(MSQD_EINVAL, "absorber width outside the box");
  if (!std::isfinite(d->r_diss_au)) return fail(MSQD_EINVAL, "r_diss not finite");
  return MSQD_OK;
}

static int fd_planes(const fdtd_desc* d) { return (d->n_freq > 0 && d->mon_k2 != 0) ? 2 : 1; }

static int check_fd(const fdtd_desc* d) {
  if (!d) return fail(MSQD_EINVAL, "fdtd_desc is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 4) return fail(MSQD_EINVAL, "grid too small");
  if (static_cast<double>(d->nx) * d->ny * d->nz > 2.0e9) return fail(MSQD_EUNSUP, "grid too large");
  if (d->nz > 65535) return fail(MSQD_EUNSUP, "nz above 65535 (one launch row of planes)");
  if (d->npml < 1 || 2 * d->npml >= d->nz) return fail(MSQD_EINVAL, "npml must satisfy 1 <= npml < nz/2");
  if (d->prec != MSQD_FP64 && d->prec != MSQD_FP32 && d->prec != MSQD_MIXED)
    return fail(MSQD_EPREC, "unknown precision");
  if (!(d->dx > 0.0) || !(d->dt > 0.0)) return fail(MSQD_EINVAL, "dx and dt must be > 0");
  if (kC0 * d->dt / d->dx > 1.0 / std::sqrt(3.0)) return fail(MSQD_EINVAL, "Courant number above 1/sqrt(3)");
  for (int m = 0; m < 4; ++m)
    if (!(d->eps_r[m] > 0.0)) return fail(MSQD_EINVAL, "eps_r must be > 0");
  if (d->metal_id < 0 || d->metal_id > 3) return fail(MSQD_EINVAL, "metal_id must be in [0, 3]");
  if (d->kappa_max < 1.0 || d->alpha_max < 0.0 || d->sigma_max_lo < 0.0 || d->sigma_max_hi < 0.0)
    return fail(MSQD_EINVAL, "bad CPML parameters");
  if (d->src_k < 1 || d->src_k >= d->nz) return fail(MSQD_EINVAL, "src_k outside the grid");
  if (d->n_freq < 0) return fail(MSQD_EINVAL, "n_freq < 0");
  if (d->n_freq > 65536) return fail(MSQD_EUNSUP, "n_freq above 65536");
  if (d->n_freq > 0) {
    if (d->mon_k <= d->npml || d->mon_k >= d->nz - d->npml)
      return fail(MSQD_EINVAL, "mon_k must be inside the interior");
    if (d->mon_every < 1) return fail(MSQD_EINVAL, "mon_every must be >= 1");
    if (d->mon_k2 != 0 && (d->mon_k2 <= d->npml || d->mon_k2 >= d->nz - d->npml))
      return fail(MSQD_EINVAL, "mon_k2 must be 0 or inside the interior");
  }
  return MSQD_OK;
}

static int check_fields(const fdtd_desc* d, const fdtd_fields* f) {
  if (!f) return fail(MSQD_EINVAL, "fdtd_fields is NULL");
  const void* ptrs[] = {f->Ex, f->Ey, f->Ez, f->Hx, f->Hy, f->Hz, f->JDx, f->JDy, f->JDz, f->psi};
  for (const void* p : ptrs) {
    if (!p) return fail(MSQD_EINVAL, "a field pointer is NULL");
    if (!aligned16(p)) return fail(MSQD_EINVAL, "field pointers must be 16-byte aligned");
  }
  if (!f->mat) return fail(MSQD_EINVAL, "material pointer is NULL");
  if (d->n_freq > 0 && (!f->dft || !aligned16(f->dft)))
    return fail(MSQD_EINVAL, "monitor buffer missing or misaligned");
  return MSQD_OK;
}

static FdArgs make_fd_args(const fdtd_desc* d, const fdtd_fields* f, const void* ws) {
  FdArgs a{};
  a.nx = d->nx;
  a.ny = d->ny;
  a.nz = d->nz;
  a.npml = d->npml;
  a.metal_id = d->metal_id;
  a.src_k = d->src_k;
  a.inv_dx = 1.0 / d->dx;
  a.cH = d->dt / kMu0;
  for (int m = 0; m < 4; ++m) a.ce[m] = d->dt / (kEps0 * d->eps_r[m]);
  const double g = d->drude_gamma, wp = d->drude_wp, dt = d->dt;
  a.alpha_d = (1.0 - g * dt / 2.0) / (1.0 + g * dt / 2.0);
  a.beta_d = kEps0 * wp * wp * dt / (1.0 + g * dt / 2.0);
  a.Ex = f->Ex;
  a.Ey = f->Ey;
  a.Ez = f->Ez;
  a.Hx = f->Hx;
  a.Hy = f->Hy;
  a.Hz = f->Hz;
  a.JDx = f->JDx;
  a.JDy = f->JDy;
  a.JDz = f->JDz;
  a.psi = f->psi;
  a.mat = f->mat;
  a.ws = static_cast<const char*>(ws);
  a.lay = fd_layout(d);
  return a;
}

static MolArgs make_mol_args(const qd_desc* d, const void* ws) {
  MolArgs a{};
  a.n_mol = d->n_mol;
  a.nj = d->j_max + 1;
  a.dr = (d->r_max - d->r_min) / d->n_r;
  a.ws = static_cast<const char*>(ws);
  a.lay = qd_layout(d->n_r, d->j_max + 1);
  a.status = reinterpret_cast<int*>(const_cast<char*>(a.ws) + a.lay.status);
  a.inv_eau = 1.0 / kEau;
  // first index with r > r_diss
  int kd = d->n_r;
  for (int k = 0; k < d->n_r; ++k) {
    if (d->r_min + k * a.dr > d->r_diss_au) {
      kd = k;
      break;
    }
  }
  a.kdiss = kd;
  // first index inside the absorber (the same test as the mask table's)
  int km = d->n_r;
  if (d->absorb_width_au > 0.0) {
    const double ra = d->r_max - d->absorb_width_au;
    for (int k = 0; k < d->n_r; ++k) {
      if (d->r_min + k * a.dr >= ra) {
        km = k;
        break;
      }
    }
  }
  a.kmask = km;
  return a;
}

static int launch_mol(const qd_desc* d, const MolArgs& a, hipStream_t s) {
  int e = 0;
  if (a.n_mol == 0) return MSQD_OK;
  if (d->basis == MSQD_BASIS_JM) {
    e = d->j_max == 1 ? launch_mol_jm(a, d->n_r, d->prec != MSQD_FP64, s)
                      : launch_mol_jmg(a, d->n_r, d->prec != MSQD_FP64, d->j_max, s);
    if (e != 0) return check_hip(static_cast<hipError_t>(e), "(j, m) molecule step launch");
    return MSQD_OK;
  }
  const size_t need = mol_lds_bytes(d->n_r, d->j_max + 1, d->prec);
  if (need > mol_lds_limit())
    return fail(MSQD_EUNSUP, "n_r x (j_max+1) too large for one workgroup's LDS in this precision (" +
                                 std::to_string(need) + " > " + std::to_string(mol_lds_limit()) + " bytes)");
  switch (d->prec) {
    case MSQD_FP64: e = launch_mol_fp64(a, d->n_r, s); break;
    case MSQD_FP32: e = launch_mol_fp32(a, d->n_r, s); break;
    default: e = launch_mol_mixed(a, d->n_r, s); break;
  }
  if (e != 0) return check_hip(static_cast<hipError_t>(e), "molecule step launch");
  return MSQD_OK;
}

__global__ void init_psi_kernel(void* psi, int n_mol, int lines, int n_r, const double* psi0,
                                double* absorbed, int is_f32) {
  const size_t per = static_cast<size_t>(lines) * n_r;
  const size_t total = per * n_mol;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t in_mol = t % per;
    const double v = (in_mol < static_cast<size_t>(n_r)) ? psi0[in_mol] : 0.0;
    if (is_f32) {
      reinterpret_cast<float2*>(psi)[t] = make_float2(static_cast<float>(v), 0.0f);
    } else {
      reinterpret_cast<double2*>(psi)[t] = make_double2(v, 0.0);
    }
    if (in_mol == 0) absorbed[t / per] = 0.0;
  }
}

}  // namespace msqd

using namespace msqd;

extern "C" {

const char* msqd_last_error(void) { return g_err.c_str(); }
int msqd_version(void) { return 200; }

static void timing_release() {
  for (hipEvent_t ev : g_timing.b) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : g_timing.e) (void)hipEventDestroy(ev);
  g_timing = MolTiming{};
}

int msqd_mol_timing_begin(int32_t max_launches) {
  if (max_launches < 1 || max_launches > (1 << 20)) return fail(MSQD_EINVAL, "max_launches outside [1, 2^20]");
  timing_release();
  g_timing.b.resize(max_launches);
  g_timing.e.resize(max_launches);
  for (int i = 0; i < max_launches; ++i) {
    hipError_t e1 = hipEventCreate(&g_timing.b[i]);
    hipError_t e2 = e1 == hipSuccess ? hipEventCreate(&g_timing.e[i]) : e1;
    if (e2 != hipSuccess) {
      g_timing.b.resize(e1 == hipSuccess ? i + 1 : i);
      g_timing.e.resize(i);
      timing_release();
      return check_hip(e2, "hipEventCreate");
    }
  }
  g_timing.armed = true;
  return MSQD_OK;
}

int msqd_mol_timing_end(double* total_ms, int32_t* n_launches) {
  if (!total_ms || !n_launches) return fail(MSQD_EINVAL, "NULL output");
  *total_ms = 0.0;
  *n_launches = 0;
  if (!g_timing.armed) return fail(MSQD_EINVAL, "molecular timing was not started on this thread");
  double sum = 0.0;
  for (int i = 0; i < g_timing.n_rec; ++i) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(g_timing.e[i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, g_timing.b[i], g_timing.e[i]);
    if (e != hipSuccess) {
      timing_release();
      return check_hip(e, "molecular launch timing");
    }
    sum += ms;
  }
  *total_ms = sum;
  *n_launches = g_timing.n_rec;
  timing_release();
  return MSQD_OK;
}

// bytes of the general (j, m) coupling tables after the common ones
static size_t qd_jmg_bytes(const qd_desc* d) {
  return (d->basis == MSQD_BASIS_JM && d->j_max >= 2) ? 8 * static_cast<size_t>(jmg_tab(d->j_max).n) : 0;
}

// dipole_readout's ensemble sums: the dipole (one component, or x, y, z in
// the (j, m) basis), the norm and the yield; their stage-one partials sit at
// the end of the workspace, after the tables
static int qd_sum_vecs(const qd_desc* d) { return (d->basis == MSQD_BASIS_JM ? 3 : 1) + 2; }
static size_t qd_tables_bytes(const qd_desc* d) { return qd_layout(d->n_r, d->j_max + 1).total + qd_jmg_bytes(d); }
static size_t qd_partials_offset(const qd_desc* d) { return align256(qd_tables_bytes(d)); }
static size_t qd_partials_bytes(const qd_desc* d) {
  return sizeof(double) * qd_sum_vecs(d) * static_cast<size_t>(sum_blocks(d->n_mol));
}

size_t qd_workspace_bytes(const qd_desc* d) {
  if (check_qd(d) != MSQD_OK) return 0;
  return qd_partials_offset(d) + qd_partials_bytes(d);
}

size_t qd_jm_tables_size(int32_t j_max) {
  return (j_max >= 2 && j_max <= kJmgMax) ? static_cast<size_t>(jmg_tab(j_max).n) : 0;
}

int qd_jm_tables(int32_t j_max, double* out, size_t n_out) {
  if (j_max < 2 || j_max > kJmgMax)
    return fail(MSQD_EUNSUP, "the general (j, m) tables exist for 2 <= j_max <= " + std::to_string(kJmgMax));
  if (!out) return fail(MSQD_EINVAL, "output pointer is NULL");
  const size_t need = qd_jm_tables_size(j_max);
  if (n_out < need) return fail(MSQD_ESHAPE, "output holds fewer than " + std::to_string(need) + " doubles");
  if (!fill_jmg_tables(j_max, out)) return fail(MSQD_EDEVICE, "eigen-decomposition did not converge");
  return MSQD_OK;
}

int qd_init(const qd_desc* d, const double* U_g, const double* U_e, const double* mu12,
            const double* psi0, void* ws, size_t ws_bytes, void* psi, double* absorbed,
            void* stream) {
  int rc = check_qd(d);
  if (rc) return rc;
  if (!U_g || !U_e || !mu12 || !psi0) return fail(MSQD_EINVAL, "host table pointer is NULL");
  if (!ws || !aligned16(ws)) return fail(MSQD_EINVAL, "workspace NULL or misaligned");
  const QdLayout L = qd_layout(d->n_r, d->j_max + 1);
  const size_t ws_need = qd_tables_bytes(d);
  if (ws_bytes < qd_partials_offset(d) + qd_partials_bytes(d)) return fail(MSQD_ESHAPE, "workspace too small");
  if (d->n_mol > 0 && (!psi || !aligned16(psi) || !absorbed))
    return fail(MSQD_EINVAL, "psi / absorbed NULL or misaligned");
  for (int k = 0; k < d->n_r; ++k)
    if (!std::isfinite(U_g[k]) || !std::isfinite(U_e[k]) || !std::isfinite(mu12[k]) || !std::isfinite(psi0[k]))
      return fail(MSQD_EINVAL, "non-finite value in the model tables");
  hipStream_t s = static_cast<hipStream_t>(stream);

  const MolTablesHost t = build_mol_tables(*d, U_g, U_e, mu12);
  std::vector<unsigned char> host(ws_need, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) { std::memcpy(host.data() + off, src, bytes); };
  const int nr = d->n_r, nj = d->j_max + 1;
  if (qd_jmg_bytes(d) > 0 && !fill_jmg_tables(d->j_max, reinterpret_cast<double*>(host.data() + L.total)))
    return fail(MSQD_EDEVICE, "(j, m) coupling tables: eigen-decomposition did not converge");
  put(L.psi0, psi0, 8 * nr);
  put(L.kin_d, t.kin.data(), 16 * nr);
  put(L.tw_d, t.tw.data(), 16 * t.tw.size());
  put(L.vph_d, t.vph.data(), 16 * t.vph.size());
  put(L.x_d, t.x.data(), 8 * nj);
  put(L.mudt_d, t.mudt.data(), 8 * nr);
  put(L.mask_d, t.mask.data(), 8 * nr);
  put(L.mu_d, t.mu.data(), 8 * nr);
  put(L.cj_d, t.cj.data(), 8 * nj);
  auto putf = [&](size_t off, const std::vector<double>& v) {
    float* dst = reinterpret_cast<float*>(host.data() + off);
    for (size_t i = 0; i < v.size(); ++i) dst[i] = static_cast<float>(v[i]);
  };
  // FP32 phase tables: the kinetic and potential phases as lifting
  // parameters (the kinetic one without its 1/n_r), the transform twiddles
  // as float pairs of modulus closest to one
  auto put_lift = [&](size_t off, const std::vector<std::complex<double>>& v, double scale) {
    float* dst = reinterpret_cast<float*>(host.data() + off);
    for (size_t i = 0; i < v.size(); ++i)
      lift_params(v[i].real() * scale, v[i].imag() * scale, &dst[2 * i], &dst[2 * i + 1]);
  };
  auto put_unit = [&](size_t off, const std::vector<std::complex<double>>& v) {
    float* dst = reinterpret_cast<float*>(host.data() + off);
    for (size_t i = 0; i < v.size(); ++i) unit_pair_f32(v[i].real(), v[i].imag(), &dst[2 * i], &dst[2 * i + 1]);
  };
  put_lift(L.kin_f, t.kin, static_cast<double>(nr));
  put_unit(L.tw_f, t.tw_f);
  {
    // the same twiddles times n_r^(-1/2), an exact power of two when log2 n_r
    // is even: the complex64 step applies the inverse transform's 1/n_r
    // through the twiddles of its two passes
    int lg = 0;
    while ((1 << lg) < nr) ++lg;
    const float sc = (lg % 2 == 0) ? std::ldexp(1.0f, -lg / 2) : 1.0f;
    const float* src = reinterpret_cast<const float*>(host.data() + L.tw_f);
    float* dst = reinterpret_cast<float*>(host.data() + L.tw_fs);
    for (size_t i = 0; i < 2 * t.tw_f.size(); ++i) dst[i] = src[i] * sc;
  }
  put_lift(L.vph_f, t.vph, 1.0);
  putf(L.x_f, t.x);
  putf(L.mudt_f, t.mudt);
  putf(L.mask_f, t.mask);
  fill_mfma_fragments(host.data() + L.tmfrag, t.tm, nj);
  {
    double* fd = reinterpret_cast<double*>(host.data() + L.tmfrag_d);
    float* ff = reinterpret_cast<float*>(host.data() + L.tmfrag_f);
    // lane l, element i owns row 4 (l/16) + i (FP32 instruction) or
    // 4 i + l/16 (FP64 instruction) of the 16-row operand blocks (entry()
    // is zero for rows or columns >= nj, kMaxNJ included)
    auto entry = [&](int row, int k) { return (row < nj && k < nj) ? t.tm[static_cast<size_t>(row) * nj + k] : 0.0; };
    // With nj <= kHalfKMaxNJ the FP32 blocks take the half-K order: operand
    // position m = 4g + i holds row 2g + i for i < 2 and nothing otherwise,
    // and element i of lane group g feeds row 2g + i (i < 2)
    const bool half = nj <= kHalfKMaxNJ;
    auto pos_row = [&](int m) { return half ? ((m & 3) < 2 ? 2 * (m >> 2) + (m & 3) : kMaxNJ) : m; };
    for (int lane = 0; lane < 64; ++lane)
      for (int i = 0; i < 4; ++i) {
        const int c = lane % 16, g = lane / 16;
        const int kf = half ? (i < 2 ? 2 * g + i : kMaxNJ) : 4 * g + i, kd = 4 * i + g;
        fd[(0 * 64 + lane) * 4 + i] = entry(c, kd);
        fd[(1 * 64 + lane) * 4 + i] = entry(kd, c);
        ff[(0 * 64 + lane) * 4 + i] = static_cast<float>(entry(pos_row(c), kf));
        ff[(1 * 64 + lane) * 4 + i] = static_cast<float>(entry(kf, pos_row(c)));
      }
  }

  MSQD_HIP(hipMemcpyAsync(ws, host.data(), ws_need, hipMemcpyHostToDevice, s));
  if (d->n_mol > 0) {
    const int lines = qd_lines(d);
    const size_t total = static_cast<size_t>(lines) * nr * d->n_mol;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(init_psi_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, psi,
                       d->n_mol, lines, nr,
                       reinterpret_cast<const double*>(static_cast<char*>(ws) + L.psi0), absorbed,
                       d->prec == MSQD_FP64 ? 0 : 1);
    MSQD_HIP(hipGetLastError());
  }
  MSQD_HIP(hipStreamSynchronize(s));
  return MSQD_OK;
}

int qd_step(const qd_desc* d, const void* ws, void* psi, const double* E_mol, double* absorbed,
            double* d_mol, int32_t n_steps, void* stream) {
  int rc = check_qd(d);
  if (rc) return rc;
  if (n_steps < 0) return fail(MSQD_EINVAL, "n_steps < 0");
  if (d->n_mol == 0 || n_steps == 0) return MSQD_OK;
  if (!ws || !psi || !E_mol || !absorbed) return fail(MSQD_EINVAL, "NULL device pointer");
  if (!aligned16(ws) || !aligned16(psi)) return fail(MSQD_EINVAL, "misaligned device pointer");
  MolArgs a = make_mol_args(d, ws);
  a.n_steps = n_steps;
  a.psi = psi;
  a.E_mol = E_mol;
  a.absorbed = absorbed;
  a.d_mol = d_mol;
  a.want_d = d_mol != nullptr;
  return launch_mol(d, a, static_cast<hipStream_t>(stream));
}

// per-molecule readouts, then (sums != NULL) their fixed-order ensemble sums
// with the stage-one partials in `partial`
static int readout_impl(const qd_desc* d, const void* ws, const void* psi, const double* absorbed,
                        double* d_mol, double* norm_mol, double* yield_mol, double* sums, double* partial,
                        hipStream_t s) {
  if (sums && (!d_mol || !norm_mol || !yield_mol))
    return fail(MSQD_EINVAL, "sums need the per-molecule d_mol, norm_mol and yield_mol they reduce");
  if (d->n_mol > 0) {
    if (!ws || !psi || !absorbed) return fail(MSQD_EINVAL, "NULL device pointer");
    if (!aligned16(ws) || !aligned16(psi)) return fail(MSQD_EINVAL, "misaligned device pointer");
    MolArgs a = make_mol_args(d, ws);
    a.n_steps = 0;
    a.psi = const_cast<void*>(psi);
    a.E_mol = nullptr;   // no step: the kernels read no field
    a.absorbed = const_cast<double*>(absorbed);
    a.d_mol = d_mol;
    a.norm_mol = norm_mol;
    a.yield_mol = yield_mol;
    a.want_d = d_mol != nullptr;
    a.want_norm = norm_mol != nullptr;
    a.want_yield = yield_mol != nullptr;
    const int rc = launch_mol(d, a, s);
    if (rc) return rc;
  }
  if (!sums) return MSQD_OK;
  SumArgs sa{};
  const int nc = qd_sum_vecs(d) - 2;
  for (int c = 0; c < nc; ++c) {
    sa.src[c] = d_mol + c;
    sa.stride[c] = nc;
  }
  sa.src[nc] = norm_mol;
  sa.src[nc + 1] = yield_mol;
  sa.stride[nc] = sa.stride[nc + 1] = 1;
  sa.nv = nc + 2;
  sa.n = d->n_mol;
  sa.partial = partial;
  sa.out = sums;
  const int e = launch_ensemble_sums(sa, s);
  return e ? check_hip(static_cast<hipError_t>(e), "ensemble sums launch") : MSQD_OK;
}

int dipole_readout(const qd_desc* d, const void* ws, const void* psi, const double* absorbed,
                   double* d_mol, double* norm_mol, double* yield_mol, double* sums, void* stream) {
  int rc = check_qd(d);
  if (rc) return rc;
  if (sums && d->n_mol > 0 && !ws) return fail(MSQD_EINVAL, "NULL workspace");
  double* partial = (sums && d->n_mol > 0)
                        ? reinterpret_cast<double*>(static_cast<char*>(const_cast<void*>(ws)) + qd_partials_offset(d))
                        : nullptr;
  return readout_impl(d, ws, psi, absorbed, d_mol, norm_mol, yield_mol, sums, partial,
                      static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------- no-allocation readout
// Stage-one partial sums of dipole_readout_noalloc live in this file-scope
// device array instead of the workspace tail: 1024 blocks of 1024 molecules
// (n_mol <= 1,048,576) times five sums, 40 KB.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in; its device address comes from hipGetSymbolAddress,
// once per device, and only that address is passed to kernels.
constexpr int kNoallocMaxBlocks = 1024;
static __device__ __align__(256) double scratch[kNoallocMaxBlocks * kMaxSumVecs];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[64];   // device address of `scratch` per device ordinal

static int noalloc_scratch(double** out) {
  int dev = 0;
  MSQD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MSQD_EUNSUP, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MSQD_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_dev[dev]);
  return MSQD_OK;
}

int dipole_readout_noalloc(const qd_desc* d, const void* ws, const void* psi, const double* absorbed,
                           double* d_mol, double* norm_mol, double* yield_mol, double* sums, void* stream) {
  int rc = check_qd(d);
  if (rc) return rc;
  double* partial = nullptr;
  if (sums) {
    if (sum_blocks(d->n_mol) > kNoallocMaxBlocks)
      return fail(MSQD_EUNSUP, "dipole_readout_noalloc: n_mol above " + std::to_string(kNoallocMaxBlocks * kSumBlock) +
                                   " (the size of its static scratch); use dipole_readout");
    rc = noalloc_scratch(&partial);
    if (rc) return rc;
  }
  return readout_impl(d, ws, psi, absorbed, d_mol, norm_mol, yield_mol, sums, partial,
                      static_cast<hipStream_t>(stream));
}

int excited_r_readout(const qd_desc* d, const void* ws, const void* psi, double* r_num, double* pop,
                      double* sums, void* stream) {
  int rc = check_qd(d);
  if (rc) return rc;
  if (d->n_mol == 0) return MSQD_OK;
  if (!ws || !psi || !r_num || !pop) return fail(MSQD_EINVAL, "NULL pointer");
  RdArgs a{};
  a.n_mol = d->n_mol;
  a.nj = qd_lines(d) / 2;   // lines per electronic state
  a.n_r = d->n_r;
  a.r_min = d->r_min;
  a.dr = (d->r_max - d->r_min) / d->n_r;
  a.psi = psi;
  a.r_num = r_num;
  a.pop = pop;
  a.sums = sums;
  const int e = launch_excited_r(a, d->prec != MSQD_FP64, static_cast<hipStream_t>(stream));
  return e ? check_hip(static_cast<hipError_t>(e), "excited-state readout launch") : MSQD_OK;
}

int msqd_check_status(const void* ws, void* stream) {
  if (!ws) return fail(MSQD_EINVAL, "workspace NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int flag = 0;
  MSQD_HIP(hipMemcpyAsync(&flag, ws, sizeof(int), hipMemcpyDeviceToHost, s));
  MSQD_HIP(hipStreamSynchronize(s));
  if (flag != 0) {
    const int zero = 0;
    MSQD_HIP(hipMemcpyAsync(const_cast<void*>(ws), &zero, sizeof(int), hipMemcpyHostToDevice, s));
    MSQD_HIP(hipStreamSynchronize(s));
    return fail(MSQD_ENONFINITE, "a molecular step produced a non-finite value");
  }
  return MSQD_OK;
}

// ------------------------------------------------------------------ FDTD
size_t fdtd_workspace_bytes(const fdtd_desc* d) {
  if (check_fd(d) != MSQD_OK) return 0;
  return fd_layout(d).total;
}

size_t fdtd_psi_bytes(const fdtd_desc* d) {
  if (check_fd(d) != MSQD_OK) return 0;
  const size_t el = d->prec == MSQD_FP64 ? 8 : 4;
  return 4 * 2 * static_cast<size_t>(d->npml) * d->ny * d->nx * el;
}

size_t fdtd_dft_bytes(const fdtd_desc* d) {
  if (check_fd(d) != MSQD_OK) return 0;
  if (d->n_freq <= 0) return 0;
  // the accumulators, then the staged samples of each plane
  const size_t plane = static_cast<size_t>(d->ny) * d->nx;
  return fd_planes(d) * (4 * static_cast<size_t>(d->n_freq) * plane * 16 + kMonRing * 4 * plane * 8);
}

static void cpml_profile(const fdtd_desc* d, double offset, std::vector<double>& b,
                         std::vector<double>& a, std::vector<double>& kinv) {
  const int nz = d->nz, np = d->npml;
  b.assign(nz, 1.0);
  a.assign(nz, 0.0);
  kinv.assign(nz, 1.0);
  for (int k = 0; k < nz; ++k) {
    const double z = k + offset;
    double depth, smax;
    if (z < np) {
      depth = (np - z) / np;
      smax = d->sigma_max_lo;
    } else if (z > nz - np) {
      depth = (z - (nz - np)) / np;
      smax = d->sigma_max_hi;
    } else {
      continue;
    }
    const double g = std::pow(depth, d->cpml_m);
    const double sig = smax * g;
    const double kap = 1.0 + (d->kappa_max - 1.0) * g;
    const double al = d->alpha_max * (1.0 - depth);
    const double bb = std::exp(-(sig / kap + al) * d->dt / kEps0);
    b[k] = bb;
    kinv[k] = 1.0 / kap;
    a[k] = sig > 0.0 ? sig * (bb - 1.0) / (sig * kap + kap * kap * al) : 0.0;
  }
}

int fdtd_init(const fdtd_desc* d, const uint8_t* mat_host, const double* freqs,
              const fdtd_fields* f, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_fd(d);
  if (rc) return rc;
  rc = check_fields(d, f);
  if (rc) return rc;
  if (!mat_host) return fail(MSQD_EINVAL, "material map is NULL");
  if (d->n_freq > 0 && !freqs) return fail(MSQD_EINVAL, "monitor frequencies missing");
  const FdLayout L = fd_layout(d);
  if (!ws || !aligned16(ws)) return fail(MSQD_EINVAL, "workspace NULL or misaligned");
  if (ws_bytes < L.total) return fail(MSQD_ESHAPE, "workspace too small");
  const size_t n = static_cast<size_t>(d->nx) * d->ny * d->nz;
  for (size_t i = 0; i < 3 * n; ++i)
    if (mat_host[i] > 3) return fail(MSQD_EINVAL, "material id above 3");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<unsigned char> host(L.total, 0);
  std::vector<double> b, a, k;
  auto put = [&](size_t off, const std::vector<double>& v) {
    std::memcpy(host.data() + off, v.data(), 8 * v.size());
  };
  auto putf = [&](size_t off, const std::vector<double>& v) {
    float* dst = reinterpret_cast<float*>(host.data() + off);
    for (size_t i = 0; i < v.size(); ++i) dst[i] = static_cast<float>(v[i]);
  };
  cpml_profile(d, 0.0, b, a, k);
  put(L.bE, b); put(L.aE, a); put(L.kE, k);
  putf(L.bEf, b); putf(L.aEf, a); putf(L.kEf, k);
  cpml_profile(d, 0.5, b, a, k);
  put(L.bH, b); put(L.aH, a); put(L.kH, k);
  putf(L.bHf, b); putf(L.aHf, a); putf(L.kHf, k);
  if (d->n_freq > 0) std::memcpy(host.data() + L.freqs, freqs, 8 * static_cast<size_t>(d->n_freq));
  MSQD_HIP(hipMemcpyAsync(ws, host.data(), L.total, hipMemcpyHostToDevice, s));
  MSQD_HIP(hipMemcpyAsync(f->mat, mat_host, 3 * n, hipMemcpyHostToDevice, s));
  const size_t el = d->prec == MSQD_FP64 ? 8 : 4;
  void* arrs[] = {f->Ex, f->Ey, f->Ez, f->Hx, f->Hy, f->Hz, f->JDx, f->JDy, f->JDz};
  for (void* p : arrs) {
    int e = launch_fill_zero(p, n * el, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "field zero fill");
  }
  int e = launch_fill_zero(f->psi, fdtd_psi_bytes(d), s);
  if (e) return check_hip(static_cast<hipError_t>(e), "CPML zero fill");
  if (d->n_freq > 0) {
    e = launch_fill_zero(f->dft, fdtd_dft_bytes(d), s);
    if (e) return check_hip(static_cast<hipError_t>(e), "monitor zero fill");
  }
  MSQD_HIP(hipStreamSynchronize(s));
  return MSQD_OK;
}

// The monitor samples of one call: staged in the ring behind the
// accumulators and folded in kMonRing at a time and at the call's last
// sample, so that every call ends with the accumulators complete; a call
// whose only sample finds the ring empty updates them directly.
struct MonBatch {
  int ns = 0;
  double tE[kMonRing], tH[kMonRing];
};

static MonArgs mon_args(const fdtd_desc* d, const fdtd_fields* f, const void* ws, int plane_index) {
  MonArgs m{};
  m.nx = d->nx;
  m.ny = d->ny;
  m.mon_k = plane_index == 0 ? d->mon_k : d->mon_k2;
  m.n_freq = d->n_freq;
  m.wdt = d->mon_every * d->dt;
  m.Ex = f->Ex;
  m.Ey = f->Ey;
  m.Hx = f->Hx;
  m.Hy = f->Hy;
  const size_t plane = static_cast<size_t>(d->ny) * d->nx;
  m.dft = f->dft + plane_index * 2 * 4 * static_cast<size_t>(d->n_freq) * plane;
  m.ring = f->dft + fd_planes(d) * 2 * 4 * static_cast<size_t>(d->n_freq) * plane +
           plane_index * static_cast<size_t>(kMonRing) * 4 * plane;
  m.freqs = reinterpret_cast<const double*>(static_cast<const char*>(ws) + fd_layout(d).freqs);
  return m;
}

// the monitor part of step n of a call whose last step is n_last
static int fd_monitor(const fdtd_desc* d, const fdtd_fields* f, const void* ws, int64_t n, int64_t n_last,
                      MonBatch& b, hipStream_t s) {
  if (d->n_freq <= 0 || (n + 1) % d->mon_every != 0) return MSQD_OK;
  const bool f32 = d->prec != MSQD_FP64;
  const bool last = n + d->mon_every > n_last;   // no further sample in this call
  const double tE = static_cast<double>(n + 1) * d->dt, tH = (static_cast<double>(n) + 0.5) * d->dt;
  const int planes = fd_planes(d);
  if (b.ns == 0 && last) {
    for (int pl = 0; pl < planes; ++pl) {
      MonArgs m = mon_args(d, f, ws, pl);
      m.tE = tE;
      m.tH = tH;
      const int e = launch_monitor(m, f32, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "monitor launch");
    }
    return MSQD_OK;
  }
  for (int pl = 0; pl < planes; ++pl) {
    MonArgs m = mon_args(d, f, ws, pl);
    m.slot = b.ns;
    const int e = launch_monitor_stage(m, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "monitor stage launch");
  }
  b.tE[b.ns] = tE;
  b.tH[b.ns] = tH;
  ++b.ns;
  if (b.ns == kMonRing || last) {
    for (int pl = 0; pl < planes; ++pl) {
      MonArgs m = mon_args(d, f, ws, pl);
      m.ns = b.ns;
      for (int i = 0; i < b.ns; ++i) {
        m.tEs[i] = b.tE[i];
        m.tHs[i] = b.tH[i];
      }
      const int e = launch_monitor_fold(m, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "monitor fold launch");
    }
    b.ns = 0;
  }
  return MSQD_OK;
}

int fdtd_step(const fdtd_desc* d, const fdtd_fields* f, const void* ws, int64_t n,
              double src_value, void* stream) {
  int rc = check_fd(d);
  if (rc) return rc;
  rc = check_fields(d, f);
  if (rc) return rc;
  if (!ws) return fail(MSQD_EINVAL, "workspace NULL");
  if (!std::isfinite(src_value)) return fail(MSQD_EINVAL, "source value not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  FdArgs a = make_fd_args(d, f, ws);
  a.src_term = -2.0 * src_value / (kEta0 * d->dx);
  const bool f32 = d->prec != MSQD_FP64;
  int e = launch_yee_h(a, f32, s);
  if (e) return check_hip(static_cast<hipError_t>(e), "H update launch");
  e = launch_yee_e(a, f32, s);
  if (e) return check_hip(static_cast<hipError_t>(e), "E update launch");
  MonBatch mb;
  return fd_monitor(d, f, ws, n, n, mb, s);
}

int flux_readout(const fdtd_desc* d, const fdtd_fields* f, double* flux, void* stream) {
  int rc = check_fd(d);
  if (rc) return rc;
  if (d->n_freq <= 0) return fail(MSQD_EINVAL, "no monitor frequencies");
  if (!f || !f->dft || !flux) return fail(MSQD_EINVAL, "NULL pointer");
  const size_t plane = 2 * 4 * static_cast<size_t>(d->n_freq) * d->ny * d->nx;  // doubles
  for (int p = 0; p < fd_planes(d); ++p) {
    const int e = launch_flux(d->nx, d->ny, d->n_freq, f->dft + p * plane, flux + p * d->n_freq,
                              static_cast<hipStream_t>(stream));
    if (e) return check_hip(static_cast<hipError_t>(e), "flux launch");
  }
  return MSQD_OK;
}

int spectra_readout(const fdtd_desc* d, const double* flux, const double* flux_ref, double* tra, void* stream) {
  int rc = check_fd(d);
  if (rc) return rc;
  if (d->n_freq <= 0) return fail(MSQD_EINVAL, "no monitor frequencies");
  if (fd_planes(d) != 2) return fail(MSQD_EINVAL, "spectra need the second detection plane (mon_k2)");
  if (!flux || !flux_ref || !tra) return fail(MSQD_EINVAL, "NULL pointer");
  const int e = launch_spectra(flux, flux + d->n_freq, flux_ref, d->n_freq, tra, static_cast<hipStream_t>(stream));
  return e ? check_hip(static_cast<hipError_t>(e), "spectra launch") : MSQD_OK;
}

// --------------------------------------------------------------- coupling
int map_build(int32_t n_mol, int32_t nx, int32_t ny, int32_t nz, uint64_t seed, int32_t slab_k0,
              int32_t slab_nk, int32_t* cell_of_mol, int32_t* occ_cell, int32_t* occ_ptr,
              int32_t* mol_perm, int32_t* n_occ) {
  if (n_mol < 0 || nx < 1 || ny < 1 || nz < 1) return fail(MSQD_EINVAL, "bad sizes");
  if (slab_nk < 1 || slab_k0 < 1 || slab_k0 + slab_nk > nz) return fail(MSQD_EINVAL, "slab outside the grid");
  if (static_cast<double>(nx) * ny * nz > 2.0e9) return fail(MSQD_EUNSUP, "grid too large");
  if (!cell_of_mol || !occ_cell || !occ_ptr || !mol_perm || !n_occ) return fail(MSQD_EINVAL, "NULL output");
  place_slab(n_mol, nx, ny, seed, slab_k0, slab_nk, cell_of_mol);
  *n_occ = build_csr(n_mol, nx * ny * nz, cell_of_mol, occ_cell, occ_ptr, mol_perm);
  return MSQD_OK;
}

int map_csr(int32_t n_mol, int32_t n_cells, const int32_t* cell_of_mol, int32_t* occ_cell,
            int32_t* occ_ptr, int32_t* mol_perm, int32_t* n_occ) {
  if (n_mol < 0 || n_cells < 1) return fail(MSQD_EINVAL, "bad sizes");
  if (!cell_of_mol || !occ_cell || !occ_ptr || !mol_perm || !n_occ) return fail(MSQD_EINVAL, "NULL pointer");
  for (int32_t m = 0; m < n_mol; ++m)
    if (cell_of_mol[m] < 0 || cell_of_mol[m] >= n_cells) return fail(MSQD_EINVAL, "cell index out of range");
  *n_occ = build_csr(n_mol, n_cells, cell_of_mol, occ_cell, occ_ptr, mol_perm);
  return MSQD_OK;
}

int map_planes(int32_t n_occ, const int32_t* occ_cell, int32_t nx, int32_t ny, int32_t nz,
               int32_t* held_k0, int32_t* held_nk) {
  if (n_occ < 1 || nx < 1 || ny < 1 || nz < 1) return fail(MSQD_EINVAL, "bad sizes");
  if (!occ_cell || !held_k0 || !held_nk) return fail(MSQD_EINVAL, "NULL pointer");
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  int64_t lo = nz, hi = -1;
  for (int32_t c = 0; c < n_occ; ++c) {
    if (occ_cell[c] < 0 || occ_cell[c] >= plane * nz) return fail(MSQD_EINVAL, "cell index out of range");
    const int64_t k = occ_cell[c] / plane;
    lo = std::min(lo, k);
    hi = std::max(hi, k);
  }
  *held_k0 = static_cast<int32_t>(lo);
  *held_nk = static_cast<int32_t>(hi - lo + 1);
  return MSQD_OK;
}

int coupled_step(const cpl_desc* d, const cpl_state* st, const double* src_values, int64_t n0,
                 int32_t n_steps, void* stream) {
  if (!d || !st) return fail(MSQD_EINVAL, "NULL descriptor or state");
  int rc = check_qd(&d->qd);
  if (rc) return rc;
  rc = check_fd(&d->fd);
  if (rc) return rc;
  rc = check_fields(&d->fd, &st->f);
  if (rc) return rc;
  if (n_steps < 0 || (n_steps > 0 && !src_values)) return fail(MSQD_EINVAL, "bad step count or source");
  const bool f32 = d->fd.prec != MSQD_FP64;
  if ((d->qd.prec == MSQD_FP64) != (d->fd.prec == MSQD_FP64))
    return fail(MSQD_EPREC, "molecule and field precision must both be FP64 or both reduced");
  if (d->n_occ < 0 || d->n_occ > d->qd.n_mol) return fail(MSQD_ESHAPE, "n_occ out of range");
  if (d->qd.n_mol > 0 && (!st->psi || !st->absorbed || !st->d_mol || !st->P_c || !st->J_mol ||
                          !st->cell_of_mol || !st->occ_cell || !st->occ_ptr || !st->mol_perm ||
                          !st->qd_ws))
    return fail(MSQD_EINVAL, "NULL coupling pointer");
  if (!st->fd_ws) return fail(MSQD_EINVAL, "NULL field workspace");
  if (d->mol_every < 0) return fail(MSQD_EINVAL, "mol_every < 0");
  if (st->psi_next) {
    if (d->qd.basis != MSQD_BASIS_M0) return fail(MSQD_EUNSUP, "psi_next (out-of-place step) needs the m = 0 basis");
    if (n_steps != 1) return fail(MSQD_EINVAL, "psi_next (out-of-place step) needs n_steps = 1");
    if (!aligned16(st->psi_next) || st->psi_next == st->psi) return fail(MSQD_EINVAL, "psi_next misaligned or equal to psi");
  }
  if (st->E_held) {
    if (!aligned16(st->E_held)) return fail(MSQD_EINVAL, "E_held misaligned");
    if (d->held_nk < 1 || d->held_k0 < 0 || d->held_k0 > d->fd.nz - d->held_nk)
      return fail(MSQD_EINVAL, "held planes outside the grid");
  }
  const int M = d->mol_every > 1 ? d->mol_every : 1;
  {
    // the molecular step must be M field steps (atomic unit of time, CODATA 2018)
    const double dt_mol_s = d->qd.dt_au * kTau;
    if (!(std::fabs(dt_mol_s - M * d->fd.dt) <= 1e-9 * M * d->fd.dt))
      return fail(MSQD_EINVAL, "qd.dt_au must equal mol_every * fd.dt (in atomic units)");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  FdArgs fa = make_fd_args(&d->fd, &st->f, st->fd_ws);
  MolArgs ma = make_mol_args(&d->qd, st->qd_ws);
  ma.n_steps = 1;
  ma.psi = st->psi;
  ma.psi_out = st->psi_next;
  ma.E_mol = nullptr;
  ma.Ex = st->f.Ex;
  ma.ex_is_float = f32 ? 1 : 0;
  ma.cell_of_mol = st->cell_of_mol;
  ma.E_out = st->E_mol;
  ma.absorbed = st->absorbed;
  ma.d_mol = st->d_mol;
  ma.want_d = 1;
  DepArgs da{};
  da.n_occ = d->n_occ;
  da.pfac = d->mol_weight * kEa0 / (d->fd.dx * d->fd.dx * d->fd.dx);
  da.inv_dt = 1.0 / (M * d->fd.dt);
  for (int m = 0; m < 4; ++m) da.ce[m] = d->fd.dt / (kEps0 * d->fd.eps_r[m]);
  da.d_mol = st->d_mol;
  da.occ_cell = st->occ_cell;
  da.occ_ptr = st->occ_ptr;
  da.mol_perm = st->mol_perm;
  da.mat = st->f.mat;
  da.P_c = st->P_c;
  da.J_mol = st->J_mol;
  da.Ex = st->f.Ex;
  da.ncomp = 1;
  if (d->qd.basis == MSQD_BASIS_JM) {
    // all three components: gathered at, and deposited on, each cell's own
    // E_x, E_y, E_z edges; P_c and J_mol are [n_occ][3]
    ma.Ey = st->f.Ey;
    ma.Ez = st->f.Ez;
    da.ncomp = 3;
    da.Ey = st->f.Ey;
    da.Ez = st->f.Ez;
  }
  da.ncells = static_cast<long>(d->fd.nx) * d->fd.ny * d->fd.nz;
  const bool held = st->E_held != nullptr;
  if (held) {
    fa.held = st->E_held;
    fa.held_k0 = d->held_k0;
    fa.held_nk = d->held_nk;
    fa.held_nc = da.ncomp;
    da.held = st->E_held;
    da.held_k0 = d->held_k0;
    da.held_nk = d->held_nk;
    da.plane = static_cast<long>(d->fd.nx) * d->fd.ny;
  }
  for (int32_t t = 0; t < n_steps; ++t)
    if (!std::isfinite(src_values[t])) return fail(MSQD_EINVAL, "source value not finite");
  if (held && n_steps > 0 && (n0 % M) != 0) {
    // between updates: the held array from the current J_mol
    da.update = 0;
    const int e = launch_deposit(da, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "held current launch");
  }
  MonBatch mb;
  for (int32_t t = 0; t < n_steps; ++t) {
    const int64_t n = n0 + t;
    const bool mol_now = (n % M) == 0;
    fa.src_term = -2.0 * src_values[t] / (kEta0 * d->fd.dx);
    int e = launch_yee_h(fa, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "H update launch");
    if (mol_now) {
      timing_mark(true, s);
      rc = launch_mol(&d->qd, ma, s);
      if (rc) return rc;
      timing_mark(false, s);
    }
    if (held) {
      // the new current goes into the held array; the E update subtracts it
      if (mol_now) {
        da.update = 1;
        e = launch_deposit(da, f32, s);
        if (e) return check_hip(static_cast<hipError_t>(e), "deposit launch");
      }
      e = launch_yee_e(fa, f32, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "E update launch");
    } else {
      e = launch_yee_e(fa, f32, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "E update launch");
      da.update = mol_now ? 1 : 0;
      e = launch_deposit(da, f32, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "deposit launch");
    }
    rc = fd_monitor(&d->fd, &st->f, st->fd_ws, n, n0 + n_steps - 1, mb, s);
    if (rc) return rc;
  }
  return MSQD_OK;
}

// ------------------------------------------------------------ Bloch emitters
static int check_bloch(const bloch_desc* d) {
  if (!d) return fail(MSQD_EINVAL, "NULL Bloch descriptor");
  if (d->n < 0) return fail(MSQD_EINVAL, "n < 0");
  if (d->prec != MSQD_FP64 && d->prec != MSQD_FP32 && d->prec != MSQD_MIXED)
    return fail(MSQD_EPREC, "unknown precision");
  const double v[] = {d->omega0_au, d->mu_au, d->gamma1_au, d->gamma2_au, d->dt_au};
  for (double x : v)
    if (!std::isfinite(x)) return fail(MSQD_EINVAL, "non-finite Bloch parameter");
  if (!(d->dt_au > 0.0)) return fail(MSQD_EINVAL, "dt_au must be positive");
  if (d->gamma1_au < 0.0 || d->gamma2_au < 0.0) return fail(MSQD_EINVAL, "negative decay rate");
  return MSQD_OK;
}

static BlochArgs make_bloch_args(const bloch_desc* d, void* state) {
  BlochArgs a{};
  a.n = d->n;
  a.w0 = d->omega0_au;
  a.mu = d->mu_au;
  a.g1 = d->gamma1_au;
  a.g2 = d->gamma2_au;
  a.dt = d->dt_au;
  a.state = state;
  a.inv_eau = 1.0 / kEau;
  return a;
}

int bloch_init(const bloch_desc* d, void* state, void* stream) {
  int rc = check_bloch(d);
  if (rc) return rc;
  if (d->n == 0) return MSQD_OK;
  if (!state || !aligned16(state)) return fail(MSQD_EINVAL, "state NULL or misaligned");
  const size_t el = d->prec == MSQD_FP64 ? 8 : 4;
  const int e = launch_fill_zero(state, 3 * static_cast<size_t>(d->n) * el, static_cast<hipStream_t>(stream));
  return e ? check_hip(static_cast<hipError_t>(e), "Bloch state fill") : MSQD_OK;
}

int bloch_step(const bloch_desc* d, void* state, const double* E, double* d_out, int32_t n_steps,
               void* stream) {
  int rc = check_bloch(d);
  if (rc) return rc;
  if (n_steps < 0) return fail(MSQD_EINVAL, "n_steps < 0");
  if (d->n == 0) return MSQD_OK;
  if (!state || !aligned16(state) || !E) return fail(MSQD_EINVAL, "state or field NULL or misaligned");
  BlochArgs a = make_bloch_args(d, state);
  a.n_steps = n_steps;
  a.E = E;
  a.d = d_out;
  const int e = launch_bloch(a, d->prec != MSQD_FP64, static_cast<hipStream_t>(stream));
  return e ? check_hip(static_cast<hipError_t>(e), "Bloch step launch") : MSQD_OK;
}

int coupled_bloch_step(const cpl_bloch_desc* d, const cpl_bloch_state* st, const double* src_values,
                       int64_t n0, int32_t n_steps, void* stream) {
  if (!d || !st) return fail(MSQD_EINVAL, "NULL descriptor or state");
  int rc = check_bloch(&d->bl);
  if (rc) return rc;
  rc = check_fd(&d->fd);
  if (rc) return rc;
  rc = check_fields(&d->fd, &st->f);
  if (rc) return rc;
  if (n_steps < 0 || (n_steps > 0 && !src_values)) return fail(MSQD_EINVAL, "bad step count or source");
  if ((d->bl.prec == MSQD_FP64) != (d->fd.prec == MSQD_FP64))
    return fail(MSQD_EPREC, "emitter and field precision must both be FP64 or both reduced");
  if (d->n_occ < 0 || d->n_occ > d->bl.n) return fail(MSQD_ESHAPE, "n_occ out of range");
  if (d->bl.n > 0 && (!st->state || !aligned16(st->state) || !st->d_mol || !st->P_c || !st->J_mol ||
                      !st->cell_of_mol || !st->occ_cell || !st->occ_ptr || !st->mol_perm))
    return fail(MSQD_EINVAL, "NULL or misaligned coupling pointer");
  if (!st->fd_ws) return fail(MSQD_EINVAL, "NULL field workspace");
  if (!(std::fabs(d->bl.dt_au * kTau - d->fd.dt) <= 1e-9 * d->fd.dt))
    return fail(MSQD_EINVAL, "bl.dt_au must equal fd.dt (in atomic units)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f32 = d->fd.prec != MSQD_FP64;
  FdArgs fa = make_fd_args(&d->fd, &st->f, st->fd_ws);
  BlochArgs ba = make_bloch_args(&d->bl, st->state);
  ba.n_steps = 1;
  ba.Ex = st->f.Ex;
  ba.ex_is_float = f32 ? 1 : 0;
  ba.cell_of_mol = st->cell_of_mol;
  ba.E_out = st->E_mol;
  ba.d = st->d_mol;
  DepArgs da{};
  da.n_occ = d->n_occ;
  da.update = 1;
  da.pfac = d->weight * kEa0 / (d->fd.dx * d->fd.dx * d->fd.dx);
  da.inv_dt = 1.0 / d->fd.dt;
  for (int m = 0; m < 4; ++m) da.ce[m] = d->fd.dt / (kEps0 * d->fd.eps_r[m]);
  da.d_mol = st->d_mol;
  da.occ_cell = st->occ_cell;
  da.occ_ptr = st->occ_ptr;
  da.mol_perm = st->mol_perm;
  da.mat = st->f.mat;
  da.P_c = st->P_c;
  da.J_mol = st->J_mol;
  da.Ex = st->f.Ex;
  da.ncomp = 1;
  da.ncells = static_cast<long>(d->fd.nx) * d->fd.ny * d->fd.nz;
  MonBatch mb;
  for (int32_t t = 0; t < n_steps; ++t) {
    const int64_t n = n0 + t;
    if (!std::isfinite(src_values[t])) return fail(MSQD_EINVAL, "source value not finite");
    fa.src_term = -2.0 * src_values[t] / (kEta0 * d->fd.dx);
    int e = launch_yee_h(fa, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "H update launch");
    e = launch_bloch(ba, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "Bloch step launch");
    e = launch_yee_e(fa, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "E update launch");
    e = launch_deposit(da, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "deposit launch");
    rc = fd_monitor(&d->fd, &st->f, st->fd_ws, n, n0 + n_steps - 1, mb, s);
    if (rc) return rc;
  }
  return MSQD_OK;
}

// ---------------------------------------------------------------- adjoint
size_t adjoint_scratch_bytes(const cpl_desc* d) {
  if (!d || check_fd(&d->fd) != MSQD_OK) return 0;
  const size_t el = d->fd.prec == MSQD_FP64 ? 8 : 4;
  return 6 * static_cast<size_t>(d->fd.nx) * d->fd.ny * d->fd.nz * el;
}

static int check_adj(const cpl_desc* d, const cpl_state* st, const cpl_adj* adj) {
  if (!d || !st || !adj) return fail(MSQD_EINVAL, "NULL descriptor, state or adjoint");
  int rc = check_qd(&d->qd);
  if (rc) return rc;
  rc = check_fd(&d->fd);
  if (rc) return rc;
  if (d->qd.prec == MSQD_MIXED || d->fd.prec == MSQD_MIXED)
    return fail(MSQD_EUNSUP, "the adjoint is provided for the FP64 and FP32 forms");
  if (d->qd.basis != MSQD_BASIS_M0) return fail(MSQD_EUNSUP, "the adjoint is provided for the m = 0 basis");
  if (d->qd.prec != d->fd.prec) return fail(MSQD_EPREC, "molecule and field precision differ");
  const fdtd_fields& f = adj->lf;
  const void* ptrs[] = {f.Ex, f.Ey, f.Ez, f.Hx, f.Hy, f.Hz, f.JDx, f.JDy, f.JDz, f.psi, adj->scratch};
  for (const void* p : ptrs)
    if (!p || !aligned16(p)) return fail(MSQD_EINVAL, "adjoint field pointer NULL or misaligned");
  if (d->qd.n_mol > 0 && (!adj->lpsi || !adj->labs || !adj->ld || !adj->lE))
    return fail(MSQD_EINVAL, "adjoint molecule pointer NULL");
  if (d->mol_every > 1 && d->qd.n_mol > 0 && d->n_occ > 0 && !adj->lJ)
    return fail(MSQD_EINVAL, "adjoint of the held current (lJ) NULL with mol_every > 1");
  if (d->n_occ > 0 && !adj->lP) return fail(MSQD_EINVAL, "adjoint polarisation pointer NULL");
  if (!st->f.mat || !st->fd_ws) return fail(MSQD_EINVAL, "forward material map or workspace NULL");
  const size_t need = mol_adj_lds_bytes(d->qd.n_r, d->qd.j_max + 1, d->qd.prec != MSQD_FP64);
  if (need > mol_lds_limit())
    return fail(MSQD_EUNSUP, "n_r x (j_max+1) too large for the adjoint molecular kernel's LDS");
  return MSQD_OK;
}

int adjoint_init_yield(const cpl_desc* d, const cpl_state* st, cpl_adj* adj, void* stream) {
  int rc = check_adj(d, st, adj);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const fdtd_desc* fd = &d->fd;
  const size_t n = static_cast<size_t>(fd->nx) * fd->ny * fd->nz;
  const size_t el = fd->prec == MSQD_FP64 ? 8 : 4;
  void* arrs[] = {adj->lf.Ex, adj->lf.Ey, adj->lf.Ez, adj->lf.Hx, adj->lf.Hy, adj->lf.Hz,
                  adj->lf.JDx, adj->lf.JDy, adj->lf.JDz};
  for (void* p : arrs) {
    const int e = launch_fill_zero(p, n * el, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "adjoint zero fill");
  }
  int e = launch_fill_zero(adj->lf.psi, fdtd_psi_bytes(fd), s);
  if (e) return check_hip(static_cast<hipError_t>(e), "adjoint CPML zero fill");
  if (d->n_occ > 0) {
    e = launch_fill_zero(adj->lP, sizeof(double) * d->n_occ, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "adjoint polarisation zero fill");
    if (d->mol_every > 1 && adj->lJ) {
      e = launch_fill_zero(adj->lJ, sizeof(double) * d->n_occ, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "adjoint current zero fill");
    }
  }
  if (d->qd.n_mol > 0) {
    const MolArgs ma = make_mol_args(&d->qd, st->qd_ws);
    e = launch_yield_adj_init(adj->lpsi, adj->labs, st->psi, d->qd.n_mol, 2 * (d->qd.j_max + 1), d->qd.n_r,
                              ma.kdiss, ma.dr, 1.0 / d->qd.n_mol, d->qd.prec != MSQD_FP64, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "adjoint objective init");
  }
  return MSQD_OK;
}

int adjoint_step(const cpl_desc* d, const cpl_state* st, const void* psi_n, void* psi_np1,
                 const double* E_mol_n, cpl_adj* adj, int64_t n, double* g_src, void* stream) {
  int rc = check_adj(d, st, adj);
  if (rc) return rc;
  if (!g_src) return fail(MSQD_EINVAL, "g_src NULL");
  if (d->qd.n_mol > 0 && (!psi_n || !E_mol_n)) return fail(MSQD_EINVAL, "recorded state NULL");
  if (psi_np1 && (!aligned16(psi_np1) || psi_np1 == psi_n)) return fail(MSQD_EINVAL, "psi_np1 misaligned or equal to psi_n");
  if (n < 0) return fail(MSQD_EINVAL, "step index < 0");
  // multi-rate coupling: the molecules stepped (by M dt) only at n % M == 0
  const int M = d->mol_every > 1 ? d->mol_every : 1;
  const bool update = (n % M) == 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool f32 = d->fd.prec != MSQD_FP64;
  FdArgs lam = make_fd_args(&d->fd, &adj->lf, st->fd_ws);
  lam.mat = st->f.mat;
  FdAdjArgs fa{lam, adj->scratch};
  CplAdjArgs ca{};
  ca.n_occ = d->n_occ;
  ca.pfac = d->mol_weight * kEa0 / (d->fd.dx * d->fd.dx * d->fd.dx);
  ca.inv_dt = 1.0 / d->fd.dt;
  ca.inv_eau = 1.0 / kEau;
  for (int m = 0; m < 4; ++m) ca.ce[m] = d->fd.dt / (kEps0 * d->fd.eps_r[m]);
  ca.occ_cell = st->occ_cell;
  ca.occ_ptr = st->occ_ptr;
  ca.mol_perm = st->mol_perm;
  ca.mat = st->f.mat;
  ca.lP = adj->lP;
  ca.ld = adj->ld;
  ca.lE = adj->lE;
  ca.lEx = adj->lf.Ex;
  ca.lJ = M > 1 ? adj->lJ : nullptr;
  ca.update = update ? 1 : 0;
  ca.inv_mdt = 1.0 / (M * d->fd.dt);
  // reverse order of the forward step: deposit, E update, molecules, gather,
  // H update; the source gradient shares the deposit's launch and the gather
  // the H update's first one
  CplAdjArgs dep = ca;
  if (d->qd.n_mol <= 0) dep.n_occ = 0;
  int e = launch_src_grad_deposit_adj(lam, 2.0 / (kEta0 * d->fd.dx), g_src, dep, f32, s);
  if (e) return check_hip(static_cast<hipError_t>(e), "source gradient and deposit adjoint launch");
  e = launch_yee_e_adj(fa, f32, s);
  if (e) return check_hip(static_cast<hipError_t>(e), "E adjoint launch");
  if (d->qd.n_mol > 0 && update) {
    if (d->n_occ == 0) {
      e = launch_fill_zero(adj->ld, sizeof(double) * d->qd.n_mol, s);
      if (e) return check_hip(static_cast<hipError_t>(e), "dipole adjoint zero fill");
    }
    const MolArgs m = make_mol_args(&d->qd, st->qd_ws);
    MolAdjArgs ma{};
    ma.n_mol = d->qd.n_mol;
    ma.nj = m.nj;
    ma.kdiss = m.kdiss;
    ma.dr = m.dr;
    ma.psi_n = psi_n;
    ma.psi_np1 = psi_np1;
    ma.E_mol = E_mol_n;
    ma.lpsi = adj->lpsi;
    ma.labs = adj->labs;
    ma.ld = adj->ld;
    ma.lE = adj->lE;
    ma.ws = m.ws;
    ma.lay = m.lay;
    e = launch_mol_adj(ma, d->qd.n_r, f32, s);
    if (e) return check_hip(static_cast<hipError_t>(e), "molecular adjoint launch");
  }
  CplAdjArgs gat = ca;
  if (!(d->qd.n_mol > 0 && update)) gat.n_occ = 0;
  e = launch_yee_h_adj(fa, gat, f32, s);
  if (e) return check_hip(static_cast<hipError_t>(e), "H adjoint launch");
  return MSQD_OK;
}

}  // extern "C"
