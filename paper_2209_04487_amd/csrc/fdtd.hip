// Yee leap-frog of Eq. (1) with the Drude current of Eq. (2), CPML along z,
// periodic x/y, soft current-sheet source, detection-plane DFT, and the
// per-cell polarisation current deposit of the molecules.
//
// Each update is a bandwidth-bound stencil: one lane per cell, x fastest so
// that neighbouring lanes touch neighbouring addresses; the +-1 neighbours in
// y and z come from cache.
#include "fdtd.h"

namespace msqd {

template <typename T>
struct FdPtr {
  T *Ex, *Ey, *Ez, *Hx, *Hy, *Hz, *JDx, *JDy, *JDz, *psi;
};

template <typename T>
__device__ __forceinline__ FdPtr<T> fd_ptrs(const FdArgs& a) {
  return {static_cast<T*>(a.Ex),  static_cast<T*>(a.Ey),  static_cast<T*>(a.Ez),
          static_cast<T*>(a.Hx),  static_cast<T*>(a.Hy),  static_cast<T*>(a.Hz),
          static_cast<T*>(a.JDx), static_cast<T*>(a.JDy), static_cast<T*>(a.JDz),
          static_cast<T*>(a.psi)};
}

// plane index of k inside the CPML auxiliary arrays, or -1 outside the layers
__device__ __forceinline__ int pml_plane(int k, int nz, int npml) {
  if (k < npml) return k;
  if (k >= nz - npml) return npml + (k - (nz - npml));
  return -1;
}

template <typename T>
__device__ __forceinline__ const T* prof(const FdArgs& a, size_t off_d, size_t off_f) {
  if constexpr (sizeof(T) == 8)
    return reinterpret_cast<const T*>(a.ws + off_d);
  else
    return reinterpret_cast<const T*>(a.ws + off_f);
}

// Launch geometry of both updates: blockIdx.y is the z plane, blockIdx.x a
// run of 256 cells of that plane in x-fastest order (so the dispatch order is
// the memory order), and the in-plane (i, j) come from 32-bit arithmetic.
struct CellIdx {
  long idx;   // linear cell index
  int i, j, k;
};
__device__ __forceinline__ bool cell_of_thread(const FdArgs& a, CellIdx& c) {
  const int plane = a.nx * a.ny;
  const int p = static_cast<int>(blockIdx.x) * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
  if (p >= plane) return false;
  c.k = static_cast<int>(blockIdx.y);
  c.j = p / a.nx;
  c.i = p - c.j * a.nx;
  c.idx = static_cast<long>(c.k) * plane + p;
  return true;
}

// Material coefficient dt/(eps0 eps_r[m]) by selects instead of an indexed
// load (a lane-dependent index into the argument block is a memory access
// that every E component would wait on).
template <typename T>
__device__ __forceinline__ T ce_select(const FdArgs& a, int m) {
  const T c0 = static_cast<T>(a.ce[0]), c1 = static_cast<T>(a.ce[1]);
  const T c2 = static_cast<T>(a.ce[2]), c3 = static_cast<T>(a.ce[3]);
  const T lo = (m & 1) ? c1 : c0, hi = (m & 1) ? c3 : c2;
  return (m & 2) ? hi : lo;
}

// The molecular current's term on E.  In the reduced precisions the term
// dt/(eps0 eps_r) J is formed in FP64 and rounded to the field precision
// before the field loses it; in FP64 the product and the subtraction take a
// single rounding (fused multiply-add).  `held` is what the held-current
// array keeps for the E update: the rounded term, or J itself in FP64.
template <typename T>
struct MolTerm;
template <>
struct MolTerm<float> {
  __device__ static __forceinline__ float held(double ce, double J) { return static_cast<float>(ce * J); }
  __device__ static __forceinline__ float apply(float e, float, float h) { return e - h; }
};
template <>
struct MolTerm<double> {
  __device__ static __forceinline__ double held(double, double J) { return J; }
  __device__ static __forceinline__ double apply(double e, double ce, double h) { return fma(-ce, h, e); }
};

// H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n, with the CPML stretching of the
// z derivatives: d/dz -> (1/kappa) d/dz + psi, psi <- b psi + a d/dz.
// Every load is issued before the first store (the arrays are distinct), so
// the loads of a cell overlap instead of waiting behind the stores.
template <typename T>
__global__ __launch_bounds__(256) void yee_h_kernel(FdArgs a) {
  CellIdx cl;
  if (!cell_of_thread(a, cl)) return;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int i = cl.i, j = cl.j, k = cl.k;
  const long idx = cl.idx;
  const long sy = nx, sz = static_cast<long>(nx) * ny;
  const long ip = (i + 1 == nx) ? idx - (nx - 1) : idx + 1;
  const long jp = (j + 1 == ny) ? idx - (ny - 1) * sy : idx + sy;
  FdPtr<T> f = fd_ptrs<T>(a);
  const T* __restrict__ Ex = f.Ex;
  const T* __restrict__ Ey = f.Ey;
  const T* __restrict__ Ez = f.Ez;
  const bool below_top = k + 1 < nz;
  const T ex = Ex[idx], ey = Ey[idx], ez = Ez[idx];
  const T ex_kp = below_top ? Ex[idx + sz] : T(0);
  const T ey_kp = below_top ? Ey[idx + sz] : T(0);
  const T ez_jp = Ez[jp], ez_ip = Ez[ip], ey_ip = Ey[ip], ex_jp = Ex[jp];
  const T hx = f.Hx[idx], hy = f.Hy[idx], hz = f.Hz[idx];
  const T inv_dx = static_cast<T>(a.inv_dx);
  const T cH = static_cast<T>(a.cH);

  const T dEz_dy = (ez_jp - ez) * inv_dx;
  const T dEz_dx = (ez_ip - ez) * inv_dx;
  T dEy_dz = (ey_kp - ey) * inv_dx;
  T dEx_dz = (ex_kp - ex) * inv_dx;
  const T dEy_dx = (ey_ip - ey) * inv_dx;
  const T dEx_dy = (ex_jp - ex) * inv_dx;

  const int kk = pml_plane(k, nz, a.npml);
  if (kk >= 0) {
    const T b = prof<T>(a, a.lay.bH, a.lay.bHf)[k];
    const T c = prof<T>(a, a.lay.aH, a.lay.aHf)[k];
    const T ki = prof<T>(a, a.lay.kH, a.lay.kHf)[k];
    const long np = 2L * a.npml * sz;
    const long o = kk * sz + (idx - static_cast<long>(k) * sz);
    T* psiHx = f.psi + 2 * np;
    T* psiHy = f.psi + 3 * np;
    const T p0 = psiHx[o], p1 = psiHy[o];
    const T phx = b * p0 + c * dEy_dz;
    const T phy = b * p1 + c * dEx_dz;
    psiHx[o] = phx;
    psiHy[o] = phy;
    dEy_dz = dEy_dz * ki + phx;
    dEx_dz = dEx_dz * ki + phy;
  }
  f.Hx[idx] = hx - cH * (dEz_dy - dEy_dz);
  f.Hy[idx] = hy - cH * (dEx_dz - dEz_dx);
  f.Hz[idx] = hz - cH * (dEy_dx - dEx_dy);
}

// Drude current (centred form of Eq. (2)) and
// E^{n+1} = E^n + dt/(eps0 eps_r) [curl H^{n+1/2} - J_D^{n+1/2} - J_src].
// E_x, E_y at k = 0 stay zero (the grid ends on tangential E = 0).
// Loads first, as in the H update.
template <typename T>
__global__ __launch_bounds__(256) void yee_e_kernel(FdArgs a) {
  CellIdx cl;
  if (!cell_of_thread(a, cl)) return;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int i = cl.i, j = cl.j, k = cl.k;
  const long idx = cl.idx;
  const long n = static_cast<long>(nx) * ny * nz;
  const long sy = nx, sz = static_cast<long>(nx) * ny;
  const long im = (i == 0) ? idx + (nx - 1) : idx - 1;
  const long jm = (j == 0) ? idx + (ny - 1) * sy : idx - sy;
  FdPtr<T> f = fd_ptrs<T>(a);
  const T* __restrict__ Hx = f.Hx;
  const T* __restrict__ Hy = f.Hy;
  const T* __restrict__ Hz = f.Hz;
  const T hx = Hx[idx], hy = Hy[idx], hz = Hz[idx];
  const T hx_km = (k > 0) ? Hx[idx - sz] : T(0);
  const T hy_km = (k > 0) ? Hy[idx - sz] : T(0);
  const T hz_jm = Hz[jm], hz_im = Hz[im], hy_im = Hy[im], hx_jm = Hx[jm];
  const uint8_t* mat = a.mat;
  const int mc[3] = {mat[idx], mat[n + idx], mat[2 * n + idx]};
  T* E[3] = {f.Ex, f.Ey, f.Ez};
  T* JD[3] = {f.JDx, f.JDy, f.JDz};
  T e0[3], jd0[3], hv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) e0[c] = E[c][idx];
#pragma unroll
  for (int c = 0; c < 3; ++c) jd0[c] = (mc[c] == a.metal_id) ? JD[c][idx] : T(0);
  // the held molecular current, on the planes that hold occupied cells (k is
  // uniform over the workgroup)
  const bool in_held = k >= a.held_k0 && k < a.held_k0 + a.held_nk;
  const long hn = static_cast<long>(a.held_nk) * sz;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    hv[c] = (in_held && c < a.held_nc) ? static_cast<const T*>(a.held)[c * hn + idx - a.held_k0 * sz] : T(0);
  const T inv_dx = static_cast<T>(a.inv_dx);

  const T dHz_dy = (hz - hz_jm) * inv_dx;
  const T dHz_dx = (hz - hz_im) * inv_dx;
  T dHy_dz = (hy - hy_km) * inv_dx;
  T dHx_dz = (hx - hx_km) * inv_dx;
  const T dHy_dx = (hy - hy_im) * inv_dx;
  const T dHx_dy = (hx - hx_jm) * inv_dx;

  const int kk = pml_plane(k, nz, a.npml);
  if (kk >= 0) {
    const T b = prof<T>(a, a.lay.bE, a.lay.bEf)[k];
    const T c = prof<T>(a, a.lay.aE, a.lay.aEf)[k];
    const T ki = prof<T>(a, a.lay.kE, a.lay.kEf)[k];
    const long np = 2L * a.npml * sz;
    const long o = kk * sz + (idx - static_cast<long>(k) * sz);
    T* psiEx = f.psi;
    T* psiEy = f.psi + np;
    const T p0 = psiEx[o], p1 = psiEy[o];
    const T pex = b * p0 + c * dHy_dz;
    const T pey = b * p1 + c * dHx_dz;
    psiEx[o] = pex;
    psiEy[o] = pey;
    dHy_dz = dHy_dz * ki + pex;
    dHx_dz = dHx_dz * ki + pey;
  }
  const T curl[3] = {dHz_dy - dHy_dz, dHx_dz - dHz_dx, dHy_dx - dHx_dy};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int m = mc[c];
    T J = T(0);
    if (m == a.metal_id) {
      const T jd = static_cast<T>(a.alpha_d) * jd0[c] + static_cast<T>(a.beta_d) * e0[c];
      JD[c][idx] = jd;
      J = jd;
    }
    if (c == 0 && k == a.src_k) J += static_cast<T>(a.src_term);
    const T ce = ce_select<T>(a, m & 3);
    T e1 = e0[c] + ce * (curl[c] - J);
    if (c < 2 && k == 0) e1 = T(0);
    // the molecular current after the update, as the separate pass applies it
    if (in_held && c < a.held_nc) e1 = MolTerm<T>::apply(e1, ce, hv[c]);
    E[c][idx] = e1;
  }
}

static dim3 yee_grid(const FdArgs& a) {
  const long plane = static_cast<long>(a.nx) * a.ny;
  return dim3(static_cast<unsigned>((plane + 255) / 256), static_cast<unsigned>(a.nz));
}

int launch_yee_h(const FdArgs& a, bool f32, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(yee_h_kernel<float>, yee_grid(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(yee_h_kernel<double>, yee_grid(a), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

int launch_yee_e(const FdArgs& a, bool f32, hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(yee_e_kernel<float>, yee_grid(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(yee_e_kernel<double>, yee_grid(a), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

// ------------------------------------------------------------- monitor
// dft layout [4][n_freq][ny][nx] complex128: E_x, E_y at t_E, and H_x, H_y
// averaged over the planes mon_k -+ 1/2 at t_H.
// Grid: (plane / 256, frequency groups of kMonFreqs).  Each thread reads the
// plane point's fields and updates the accumulators of its group's
// frequencies: all of the group's loads are issued before its stores, and
// the frequency axis spreads the update over enough workgroups to fill the
// chip on small planes.
// Within one call the samples are staged (monitor_stage_kernel) and folded
// into the accumulators up to kMonRing at a time (monitor_fold_kernel): the
// accumulators, 4 n_freq complex values per point against 4 sample values,
// are then read and written once per batch.  Each accumulator takes the same
// fused multiply-adds in the same order either way.
constexpr int kMonFreqs = 4;

// the four sampled values of plane point p
template <typename T>
__device__ __forceinline__ void mon_values(const MonArgs& a, long plane, long p, double val[4]) {
  const long o = static_cast<long>(a.mon_k) * plane + p;
  val[0] = static_cast<const T*>(a.Ex)[o];
  val[1] = static_cast<const T*>(a.Ey)[o];
  val[2] = 0.5 * (static_cast<double>(static_cast<const T*>(a.Hx)[o - plane]) + static_cast<const T*>(a.Hx)[o]);
  val[3] = 0.5 * (static_cast<double>(static_cast<const T*>(a.Hy)[o - plane]) + static_cast<const T*>(a.Hy)[o]);
}

// cos and sin of w_f t_E and w_f t_H, times the weight
__device__ __forceinline__ void mon_phases(const MonArgs& a, int f, double tE, double tH, double* ph) {
  double s, c;
  sincos(a.freqs[f] * tE, &s, &c);
  ph[0] = c * a.wdt;
  ph[1] = s * a.wdt;
  sincos(a.freqs[f] * tH, &s, &c);
  ph[2] = c * a.wdt;
  ph[3] = s * a.wdt;
}

// accumulator c of frequency f at point p
__device__ __forceinline__ long mon_acc(const MonArgs& a, int c, int f, long plane, long p) {
  return (static_cast<long>(c) * a.n_freq + f) * plane + p;
}

__device__ __forceinline__ void mon_add(double2& w, double v, const double* ph, int c) {
  w.x = fma(v, ph[c < 2 ? 0 : 2], w.x);
  w.y = fma(v, ph[c < 2 ? 1 : 3], w.y);
}

template <typename T>
__global__ __launch_bounds__(256) void monitor_kernel(MonArgs a) {
  __shared__ double ph[kMonFreqs][4];
  const int f0 = static_cast<int>(blockIdx.y) * kMonFreqs;
  const int nf = min(kMonFreqs, a.n_freq - f0);
  if (threadIdx.x < nf) mon_phases(a, f0 + threadIdx.x, a.tE, a.tH, ph[threadIdx.x]);
  __syncthreads();
  const long plane = static_cast<long>(a.nx) * a.ny;
  const long p = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= plane) return;
  double val[4];
  mon_values<T>(a, plane, p, val);
  double2* acc = reinterpret_cast<double2*>(a.dft);
  double2 z[kMonFreqs][4];
#pragma unroll
  for (int fi = 0; fi < kMonFreqs; ++fi) {
    if (fi < nf) {
#pragma unroll
      for (int c = 0; c < 4; ++c) z[fi][c] = acc[mon_acc(a, c, f0 + fi, plane, p)];
    }
  }
#pragma unroll
  for (int fi = 0; fi < kMonFreqs; ++fi) {
    if (fi < nf) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        mon_add(z[fi][c], val[c], ph[fi], c);
        acc[mon_acc(a, c, f0 + fi, plane, p)] = z[fi][c];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void monitor_stage_kernel(MonArgs a) {
  const long plane = static_cast<long>(a.nx) * a.ny;
  const long p = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= plane) return;
  double val[4];
  mon_values<T>(a, plane, p, val);
#pragma unroll
  for (int c = 0; c < 4; ++c) a.ring[(static_cast<long>(a.slot) * 4 + c) * plane + p] = val[c];
}

__global__ __launch_bounds__(256) void monitor_fold_kernel(MonArgs a) {
  __shared__ double ph[kMonRing][kMonFreqs][4];
  const int f0 = static_cast<int>(blockIdx.y) * kMonFreqs;
  const int nf = min(kMonFreqs, a.n_freq - f0);
  const int ns = a.ns;
  if (threadIdx.x < kMonRing * kMonFreqs) {
    const int sl = threadIdx.x / kMonFreqs, fi = threadIdx.x % kMonFreqs;
    if (sl < ns && fi < nf) mon_phases(a, f0 + fi, a.tEs[sl], a.tHs[sl], ph[sl][fi]);
  }
  __syncthreads();
  const long plane = static_cast<long>(a.nx) * a.ny;
  const long p = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= plane) return;
  double2* acc = reinterpret_cast<double2*>(a.dft);
  double2 z[kMonFreqs][4];
#pragma unroll
  for (int fi = 0; fi < kMonFreqs; ++fi) {
    if (fi < nf) {
#pragma unroll
      for (int c = 0; c < 4; ++c) z[fi][c] = acc[mon_acc(a, c, f0 + fi, plane, p)];
    }
  }
  for (int sl = 0; sl < ns; ++sl) {
    double val[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) val[c] = a.ring[(static_cast<long>(sl) * 4 + c) * plane + p];
#pragma unroll
    for (int fi = 0; fi < kMonFreqs; ++fi) {
      if (fi < nf) {
#pragma unroll
        for (int c = 0; c < 4; ++c) mon_add(z[fi][c], val[c], ph[sl][fi], c);
      }
    }
  }
#pragma unroll
  for (int fi = 0; fi < kMonFreqs; ++fi) {
    if (fi < nf) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[mon_acc(a, c, f0 + fi, plane, p)] = z[fi][c];
    }
  }
}

static dim3 mon_grid(const MonArgs& a) {
  const long plane = static_cast<long>(a.nx) * a.ny;
  return dim3(static_cast<unsigned>((plane + 255) / 256),
              static_cast<unsigned>((a.n_freq + kMonFreqs - 1) / kMonFreqs));
}

int launch_monitor(const MonArgs& a, bool f32, hipStream_t s) {
  if (a.n_freq <= 0) return 0;
  if (f32)
    hipLaunchKernelGGL(monitor_kernel<float>, mon_grid(a), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(monitor_kernel<double>, mon_grid(a), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

int launch_monitor_stage(const MonArgs& a, bool f32, hipStream_t s) {
  if (a.n_freq <= 0) return 0;
  if (a.slot < 0 || a.slot >= kMonRing) return static_cast<int>(hipErrorInvalidValue);
  const long plane = static_cast<long>(a.nx) * a.ny;
  const dim3 grid(static_cast<unsigned>((plane + 255) / 256));
  if (f32)
    hipLaunchKernelGGL(monitor_stage_kernel<float>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(monitor_stage_kernel<double>, grid, dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

int launch_monitor_fold(const MonArgs& a, hipStream_t s) {
  if (a.n_freq <= 0 || a.ns <= 0) return 0;
  if (a.ns > kMonRing) return static_cast<int>(hipErrorInvalidValue);
  hipLaunchKernelGGL(monitor_fold_kernel, mon_grid(a), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

// one workgroup per frequency; fixed-order tree sum over the plane
__global__ __launch_bounds__(256) void flux_kernel(int plane, int n_freq, const double2* dft,
                                                   double* flux) {
  __shared__ double red[256];
  const int f = blockIdx.x;
  const double2* Ex = dft + (0L * n_freq + f) * plane;
  const double2* Ey = dft + (1L * n_freq + f) * plane;
  const double2* Hx = dft + (2L * n_freq + f) * plane;
  const double2* Hy = dft + (3L * n_freq + f) * plane;
  double s = 0.0;
  for (int p = threadIdx.x; p < plane; p += blockDim.x) {
    // 1/2 Re(Ex conj(Hy) - Ey conj(Hx))
    s += 0.5 * ((Ex[p].x * Hy[p].x + Ex[p].y * Hy[p].y) - (Ey[p].x * Hx[p].x + Ey[p].y * Hx[p].y));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) flux[f] = red[0] / plane;
}

int launch_flux(int nx, int ny, int n_freq, const double* dft, double* flux, hipStream_t s) {
  hipLaunchKernelGGL(flux_kernel, dim3(n_freq), dim3(256), 0, s, nx * ny, n_freq,
                     reinterpret_cast<const double2*>(dft), flux);
  return static_cast<int>(hipGetLastError());
}

// ------------------------------------------------- polarisation current
// Per occupied cell: P^{n+1} = (w e a0 / dx^3) sum_{i in cell} d_i in CSR
// order, J = (P^{n+1} - P^n)/dt_mol, and E_x at the cell loses
// dt/(eps0 eps_r) J.  Between molecular updates (multi-rate coupling) only
// the held J is applied.  With a held array the term (MolTerm) is stored
// there for the E update to apply (update = 0 then rebuilds the array from
// J_mol), and a cell outside the held planes sets its E component to NaN.
template <typename T>
__global__ __launch_bounds__(256) void deposit_kernel(DepArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_occ) return;
  const int nc = a.ncomp;
  const int cell = a.occ_cell[c];
  void* fld[3] = {a.Ex, a.Ey, a.Ez};
  // the cell's loads before its first store: the material bytes may alias
  // any array, so a load after a store would wait on it
  int mk[3];
  double pj[3];   // P_c before the update, or the held J_mol
  T e_old[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= nc) break;
    mk[k] = a.mat[static_cast<size_t>(k) * a.ncells + cell] & 3;
    pj[k] = a.update ? a.P_c[static_cast<size_t>(c) * nc + k] : a.J_mol[static_cast<size_t>(c) * nc + k];
    e_old[k] = a.held ? T(0) : static_cast<const T*>(fld[k])[cell];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k >= nc) break;
    double J;
    if (a.update) {
      double s = 0.0;
      const int b = a.occ_ptr[c], e = a.occ_ptr[c + 1];
      for (int t = b; t < e; ++t) s += a.d_mol[static_cast<size_t>(a.mol_perm[t]) * nc + k];
      const double p_new = s * a.pfac;
      J = (p_new - pj[k]) * a.inv_dt;
      a.P_c[static_cast<size_t>(c) * nc + k] = p_new;
      a.J_mol[static_cast<size_t>(c) * nc + k] = J;
    } else {
      J = pj[k];
    }
    const int m = mk[k];
    T* E = static_cast<T*>(fld[k]);
    const T h = MolTerm<T>::held(a.ce[m], J);
    if (a.held) {
      const long kc = cell / a.plane;
      if (kc >= a.held_k0 && kc < a.held_k0 + a.held_nk)
        static_cast<T*>(a.held)[(static_cast<long>(k) * a.held_nk + kc - a.held_k0) * a.plane +
                                (cell - kc * a.plane)] = h;
      else
        E[cell] = __builtin_nan("");
    } else {
      E[cell] = MolTerm<T>::apply(e_old[k], static_cast<T>(a.ce[m]), h);
    }
  }
}

int launch_deposit(const DepArgs& a, bool f32, hipStream_t s) {
  if (a.n_occ <= 0) return 0;
  const int blocks = (a.n_occ + 255) / 256;
  if (f32)
    hipLaunchKernelGGL(deposit_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(deposit_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

// ------------------------------------------------------------- zero fill
__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* p, size_t n16, unsigned char* tail,
                                                        size_t ntail) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t t = i; t < n16; t += stride) p[t] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

int launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return 0;
  const size_t n16 = bytes / 16;
  unsigned char* tail = static_cast<unsigned char*>(p) + n16 * 16;
  const size_t ntail = bytes - n16 * 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(p), n16, tail, ntail);
  return static_cast<int>(hipGetLastError());
}

}  // namespace msqd
