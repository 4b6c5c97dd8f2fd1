// Reverse-mode (adjoint) kernels of the coupled step: the exact transpose of
// every linear factor (Yee curls with their CPML recursions, the Drude
// recurrence, the source sheet, the per-cell dipole sum and the field
// gather), and the adjoint of the molecular split-operator step, including
// the derivative of the dipole-coupling rotation with respect to the field.
//
// Conventions: for a complex state psi the adjoint is
// lambda = dY/dRe(psi) + i dY/dIm(psi), so a complex-linear factor U maps
// lambda' to U^H lambda'.
#include "adjoint.h"
#include "mol_impl.h"

namespace msqd {

// ------------------------------------------------------------ molecules
// The coupling and its adjoint on the matrix cores, in the working
// precision (16x16x4 instructions, as the forward FP32 and FP64 forms), one
// wavefront per tile of 16 radial points.  A holds chi (the coupling's input)
// and B, on entry, the adjoint at its output; lane l works on radial point
// l%16 and the J (or node) rows MfmaK4<T>::row(l/16, i).  frag: [2][64][4],
// block 0 T and block 1 T^T in operand order, zero outside nj; x: the nodes.
//
// Forward (segment recompute): B = T^T R(phi) T A.
// Adjoint: Phi = T chi, Phi' = R(phi) Phi, Lambda = T lambda_out;
//   dY/dE += sum_{k,r} mu12(r) x_k dt (-Im[conj(L_g) Phi'_e + conj(L_e) Phi'_g]);
//   lambda_in = T^T R(-phi) Lambda -> B.
// Returns this lane's share of dY/dE (zero for the forward).
// A's rows are LSA elements apart (the LDS line stride, or N_r for chi in
// device memory), B's LS.  KH: N_J <= kHalfKMaxNJ, two of the four K
// instructions per product, rows as in the forward step (mf_row).
template <typename T, int NR, bool ADJ, int LSA, bool KH>
__device__ __forceinline__ double coupling_adj_mfma(const cx<T>* A, cx<T>* B, int LS, int nj,
                                                    const T* __restrict__ frag, const T* __restrict__ x,
                                                    const T* __restrict__ mudt, T E) {
  typedef typename MfmaK4<T>::acc acc_t;
  constexpr int NK = KH ? 2 : 4;
  const int lane = fresh_lane();
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nwaves = (blockDim.x + 63) >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  T Tf[4], Tt[4], xk[4];
  int rows[4], og[4], oe[4], oga[4], oea[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rows[i] = i < NK ? mf_row<T, KH>(grp, i) : kMaxNJ;
    Tf[i] = frag[(0 * 64 + lane) * 4 + i];
    Tt[i] = frag[(1 * 64 + lane) * 4 + i];
    xk[i] = (rows[i] < nj) ? x[rows[i]] : T(0);
    // loads of rows J >= nj read row nj - 1 instead: T is zero in those
    // columns, so the (finite) values read there are multiplied by zero
    const int Jc = rows[i] < nj ? rows[i] : nj - 1;
    og[i] = Jc * LS;
    oe[i] = (nj + Jc) * LS;
    oga[i] = Jc * LSA;
    oea[i] = (nj + Jc) * LSA;
  }
  double grad = 0.0;
  const acc_t z = {T(0), T(0), T(0), T(0)};
#pragma unroll 1
  for (int tile = wave; tile * 16 < NR; tile += nwaves) {
    const int r = tile * 16 + col;
    // chi (and lambda_out) rows of this lane at radial point r
    acc_t agr = z, agi = z, aer = z, aei = z, bgr = z, bgi = z, ber = z, bei = z;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const cx<T> g = A[oga[i] + r], e = A[oea[i] + r];
      agr[i] = g.x; agi[i] = g.y; aer[i] = e.x; aei[i] = e.y;
      if constexpr (ADJ) {
        const cx<T> lg = B[og[i] + r], le = B[oe[i] + r];
        bgr[i] = lg.x; bgi[i] = lg.y; ber[i] = le.x; bei[i] = le.y;
      }
    }
    acc_t Pgr = z, Pgi = z, Per = z, Pei = z, Lgr = z, Lgi = z, Ler = z, Lei = z;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      Pgr = MfmaK4<T>::mma(Tf[i], agr[i], Pgr);
      Pgi = MfmaK4<T>::mma(Tf[i], agi[i], Pgi);
      Per = MfmaK4<T>::mma(Tf[i], aer[i], Per);
      Pei = MfmaK4<T>::mma(Tf[i], aei[i], Pei);
      if constexpr (ADJ) {
        Lgr = MfmaK4<T>::mma(Tf[i], bgr[i], Lgr);
        Lgi = MfmaK4<T>::mma(Tf[i], bgi[i], Lgi);
        Ler = MfmaK4<T>::mma(Tf[i], ber[i], Ler);
        Lei = MfmaK4<T>::mma(Tf[i], bei[i], Lei);
      }
    }
    MfmaK4<T>::settle(Pgr, Pgi, Per, Pei);
    if constexpr (ADJ) MfmaK4<T>::settle(Lgr, Lgi, Ler, Lei);
    const T md = mudt[r] * E;
    T sn[4], vs[4];
    sin_vers_tile<NR>(md, xk, sn, vs);
    double gl = 0.0;
    acc_t Ogr = z, Ogi = z, Oer = z, Oei = z;   // the operand of the T^T product
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const T c = T(1) - vs[i];
      // Phi' = R(phi) Phi: [c Pg + i s Pe, i s Pg + c Pe]
      const T qgr = c * Pgr[i] - sn[i] * Pei[i], qgi = c * Pgi[i] + sn[i] * Per[i];
      const T qer = c * Per[i] - sn[i] * Pgi[i], qei = c * Pei[i] + sn[i] * Pgr[i];
      if constexpr (ADJ) {
        // -Im[conj(L_g) Q_e + conj(L_e) Q_g]
        const double im = static_cast<double>(Lgr[i] * qei - Lgi[i] * qer) +
                          static_cast<double>(Ler[i] * qgi - Lei[i] * qgr);
        gl -= static_cast<double>(xk[i]) * im;
        // R(-phi) Lambda: [c L_g - i s L_e, -i s L_g + c L_e]
        Ogr[i] = c * Lgr[i] + sn[i] * Lei[i];
        Ogi[i] = c * Lgi[i] - sn[i] * Ler[i];
        Oer[i] = c * Ler[i] + sn[i] * Lgi[i];
        Oei[i] = c * Lei[i] - sn[i] * Lgr[i];
      } else {
        Ogr[i] = qgr; Ogi[i] = qgi; Oer[i] = qer; Oei[i] = qei;
      }
    }
    if constexpr (ADJ) grad += static_cast<double>(mudt[r]) * gl;
    acc_t cgr = z, cgi = z, cer = z, cei = z;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      cgr = MfmaK4<T>::mma(Tt[i], Ogr[i], cgr);
      cgi = MfmaK4<T>::mma(Tt[i], Ogi[i], cgi);
      cer = MfmaK4<T>::mma(Tt[i], Oer[i], cer);
      cei = MfmaK4<T>::mma(Tt[i], Oei[i], cei);
    }
    MfmaK4<T>::settle(cgr, cgi, cer, cei);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      if (rows[i] < nj) {
        B[og[i] + r] = {cgr[i], cgi[i]};
        B[oe[i] + r] = {cer[i], cei[i]};
      }
    }
  }
  return grad;
}

// chi, the coupling's input, through device memory (over psi^{n+1}, which
// the reverse sweep no longer needs) instead of a second LDS buffer
template <typename T>
constexpr bool adj_chi_in_device_memory(bool next) { return next && sizeof(T) == 8; }

// NEXT: the state after the step (psi^{n+1} = m psi_pre) is given, so the
// recompute stops at chi = V K psi; otherwise the whole forward step is
// recomputed to obtain psi_pre.
// KH: N_J <= kHalfKMaxNJ (two of the four K instructions per product),
// chosen at launch so that a kernel holds one contraction path.
template <typename T, int NR, bool NEXT, bool KH>
__global__ __launch_bounds__(512) void mol_adj_kernel(MolAdjArgs a) {
  constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2;
  constexpr int LS = line_stride<NR, T>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int nj = a.nj;
  const int L = 2 * nj;
  // LDS: B (the lines) and A (chi).  complex128 with psi^{n+1} given keeps
  // chi in device memory instead (below): a molecule then needs half the LDS
  // and four instead of two share a CU, 18% faster for the FP64 gradient; in
  // complex64 the device-memory round trip of chi measured 4% slower than the
  // LDS copy, so chi stays in LDS there.
  constexpr bool CHI_DEV = adj_chi_in_device_memory<T>(NEXT);
  cx<T>* B = reinterpret_cast<cx<T>*>(smem);
  cx<T>* A = B + L * LS;
  double* red = reinterpret_cast<double*>(smem + (CHI_DEV ? 1 : 2) * sizeof(cx<T>) * L * LS);
  const int mol = blockIdx.x;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int line = tid / R2;
  const int q = tid - line * R2;
  const bool active = line < L;
  const int s_of_line = line / (nj > 0 ? nj : 1);
  const int J_of_line = line - s_of_line * nj;

  const char* ws = a.ws;
  const bool dbl = sizeof(T) == 8;
  const cx<T>* kin = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.kin_d : a.lay.kin_f));
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.tw_d : a.lay.tw_f));
  const cx<T>* vph = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.vph_d : a.lay.vph_f));
  const T* frag = reinterpret_cast<const T*>(ws + (dbl ? a.lay.tmfrag_d : a.lay.tmfrag_f));
  const T* xk = reinterpret_cast<const T*>(ws + (dbl ? a.lay.x_d : a.lay.x_f));
  const T* mudt = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mudt_d : a.lay.mudt_f));
  const T* mask = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mask_d : a.lay.mask_f));
  const double* mu = reinterpret_cast<const double*>(ws + a.lay.mu_d);
  const double* cj = reinterpret_cast<const double*>(ws + a.lay.cj_d);

  const T E = static_cast<T>(a.E_mol[mol]);
  const size_t base = static_cast<size_t>(mol) * L * NR;
  const cx<T>* psi = reinterpret_cast<const cx<T>*>(a.psi_n) + base;
  cx<T>* lpsi = reinterpret_cast<cx<T>*>(a.lpsi) + base;
  cx<T>* slot = B + line * LS;
  const int loff = line * NR + q;

  // ---- forward recompute: chi = V K psi; psi_pre = K V C(chi), or
  // psi^{n+1} = m psi_pre read back (v then holds psi^{n+1})
  cx<T> v[R1];
  cx<T>* chi_g = reinterpret_cast<cx<T>*>(a.psi_np1) + base;   // CHI_DEV: chi replaces psi^{n+1} here
  if (active) {
#pragma unroll
    for (int p = 0; p < R1; ++p) v[p] = psi[loff + R2 * p];
    kinetic_half<T, NR>(v, slot, q, kin, tw);
#pragma unroll
    for (int p = 0; p < R1; ++p) v[p] = phase_mul(v[p], vph[loff + R2 * p]);
    if constexpr (!CHI_DEV) {
#pragma unroll
      for (int p = 0; p < R1; ++p) A[line * LS + q + R2 * p] = v[p];
    }
  }
  if constexpr (CHI_DEV) {
    // psi^{n+1} into this line's LDS row (the transform above is done with
    // it), then chi over psi^{n+1} in device memory: each lane reads an
    // element before it writes it, and only this workgroup touches this
    // molecule's rows
    if (active) {
#pragma unroll
      for (int p = 0; p < R1; ++p) B[line * LS + q + R2 * p] = chi_g[loff + R2 * p];
#pragma unroll
      for (int p = 0; p < R1; ++p) chi_g[loff + R2 * p] = v[p];
#pragma unroll
      for (int p = 0; p < R1; ++p) v[p] = B[line * LS + q + R2 * p];
    }
    __syncthreads();
  } else if constexpr (NEXT) {
    const cx<T>* nxt = chi_g;
    if (active) {
#pragma unroll
      for (int p = 0; p < R1; ++p) {
        v[p] = nxt[loff + R2 * p];
        B[line * LS + q + R2 * p] = v[p];
      }
    }
    __syncthreads();
  } else {
    __syncthreads();
    coupling_adj_mfma<T, NR, false, LS, KH>(A, B, LS, nj, frag, xk, mudt, E);
    __syncthreads();
    if (active) {
#pragma unroll
      for (int p = 0; p < R1; ++p) v[p] = phase_mul(B[line * LS + q + R2 * p], vph[loff + R2 * p]);
      kinetic_half<T, NR>(v, slot, q, kin, tw);       // v = psi_pre (before the absorber)
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int p = 0; p < R1; ++p) B[line * LS + q + R2 * p] = cscale(v[p], mask[q + R2 * p]);
    }
    __syncthreads();
  }

  // ---- reverse: dipole and absorber terms, then K^H V^H
  const double ld = a.ld ? a.ld[mol] : 0.0;
  const double lab = a.labs[mol];
  cx<T> lam[R1];
  if (active) {
    const int sb = 1 - s_of_line;
    const T cjm = (J_of_line > 0) ? static_cast<T>(cj[J_of_line - 1]) : T(0);
    const T cjp = (J_of_line + 1 < nj) ? static_cast<T>(cj[J_of_line]) : T(0);
    const T fd = static_cast<T>(2.0 * a.dr * ld);
    const T fa = static_cast<T>(2.0 * a.dr * lab);
#pragma unroll
    for (int p = 0; p < R1; ++p) {
      const int r = q + R2 * p;
      cx<T> l = lpsi[loff + R2 * p];
      // D psi' with D = mu12(r) <J|cos|J'> sigma_x
      cx<T> dpsi = {T(0), T(0)};
      if (J_of_line > 0) dpsi = dpsi + cscale(B[(sb * nj + J_of_line - 1) * LS + r], cjm);
      if (J_of_line + 1 < nj) dpsi = dpsi + cscale(B[(sb * nj + J_of_line + 1) * LS + r], cjp);
      l = l + cscale(dpsi, fd * static_cast<T>(mu[r]));
      const T m = mask[r];
      // absorber term 2 dr labs (1 - m^2) psi_pre, with psi_pre = psi^{n+1} / m
      // when the state after the step was given (m > 0 on the periodic grid)
      const T wa = NEXT ? (T(1) - m * m) / m : (T(1) - m * m);
      l = cscale(l, m) + cscale(v[p], fa * wa);
      lam[p] = l;
    }
  }
  __syncthreads();
  if (active) {
    kinetic_half<T, NR, true>(lam, slot, q, kin, tw);
#pragma unroll
    for (int p = 0; p < R1; ++p) B[line * LS + q + R2 * p] = phase_mul_conj(lam[p], vph[loff + R2 * p]);
  }
  __syncthreads();
  double grad;
  if constexpr (CHI_DEV)
    grad = coupling_adj_mfma<T, NR, true, NR, KH>(chi_g, B, LS, nj, frag, xk, mudt, E);
  else
    grad = coupling_adj_mfma<T, NR, true, LS, KH>(A, B, LS, nj, frag, xk, mudt, E);
  __syncthreads();
  if (active) {
#pragma unroll
    for (int p = 0; p < R1; ++p) lam[p] = phase_mul_conj(B[line * LS + q + R2 * p], vph[loff + R2 * p]);
  }
  __syncthreads();
  if (active) {
    kinetic_half<T, NR, true>(lam, slot, q, kin, tw);
#pragma unroll
    for (int p = 0; p < R1; ++p) lpsi[loff + R2 * p] = lam[p];
  }
  double sums[4] = {grad, 0.0, 0.0, 0.0};
  block_sum4(sums, red);
  if (tid == 0) a.lE[mol] = sums[0];
}

// LDS per workgroup: two line buffers, or one where chi goes through device
// memory
static size_t adj_lds_bytes(int n_r, int nj, bool f32, bool next) {
  const size_t el = f32 ? 8 : 16;
  const int r2 = n_r / fft_r1(n_r, static_cast<int>(el / 2));
  const bool one = f32 ? adj_chi_in_device_memory<float>(next) : adj_chi_in_device_memory<double>(next);
  return (one ? 1 : 2) * el * static_cast<size_t>(2 * nj) * (n_r + r2) + 16 * 4 * sizeof(double);
}
size_t mol_adj_lds_bytes(int n_r, int nj, bool f32) { return adj_lds_bytes(n_r, nj, f32, false); }

template <typename T, int NR, bool NEXT, bool KH>
static int launch_mol_adj_n(const MolAdjArgs& a, hipStream_t s) {
  constexpr int R2 = FftShape<NR, T>::R2;
  const int L = 2 * a.nj;
  int threads = ((L * R2 + 63) / 64) * 64;
  if (threads < 64) threads = 64;
  const size_t shm = adj_lds_bytes(NR, a.nj, sizeof(T) == 4, NEXT);
  static std::atomic<unsigned long long> lds_set{0};
  if (shm > 64 * 1024) {
    const hipError_t e = allow_large_lds(reinterpret_cast<const void*>(&mol_adj_kernel<T, NR, NEXT, KH>), lds_set);
    if (e != hipSuccess) return static_cast<int>(e);
  }
  hipLaunchKernelGGL((mol_adj_kernel<T, NR, NEXT, KH>), dim3(a.n_mol), dim3(threads), shm, s, a);
  return static_cast<int>(hipGetLastError());
}

template <typename T, int NR>
static int launch_mol_adj_t(const MolAdjArgs& a, hipStream_t s) {
  if (a.nj <= kHalfKMaxNJ)
    return a.psi_np1 ? launch_mol_adj_n<T, NR, true, true>(a, s) : launch_mol_adj_n<T, NR, false, true>(a, s);
  return a.psi_np1 ? launch_mol_adj_n<T, NR, true, false>(a, s) : launch_mol_adj_n<T, NR, false, false>(a, s);
}

int launch_mol_adj(const MolAdjArgs& a, int n_r, bool f32, hipStream_t s) {
  if (f32) {
    switch (n_r) {
      case 64: return launch_mol_adj_t<float, 64>(a, s);
      case 128: return launch_mol_adj_t<float, 128>(a, s);
      case 256: return launch_mol_adj_t<float, 256>(a, s);
      case 512: return launch_mol_adj_t<float, 512>(a, s);
      default: break;
    }
  } else {
    switch (n_r) {
      case 64: return launch_mol_adj_t<double, 64>(a, s);
      case 128: return launch_mol_adj_t<double, 128>(a, s);
      case 256: return launch_mol_adj_t<double, 256>(a, s);
      case 512: return launch_mol_adj_t<double, 512>(a, s);
      default: break;
    }
  }
  return static_cast<int>(hipErrorInvalidValue);
}

// ----------------------------------------------------------------- fields
template <typename T>
struct AdjPtr {
  T *Ex, *Ey, *Ez, *Hx, *Hy, *Hz, *JDx, *JDy, *JDz, *psi;
};
template <typename T>
__device__ __forceinline__ AdjPtr<T> adj_ptrs(const FdArgs& a) {
  return {static_cast<T*>(a.Ex),  static_cast<T*>(a.Ey),  static_cast<T*>(a.Ez),
          static_cast<T*>(a.Hx),  static_cast<T*>(a.Hy),  static_cast<T*>(a.Hz),
          static_cast<T*>(a.JDx), static_cast<T*>(a.JDy), static_cast<T*>(a.JDz),
          static_cast<T*>(a.psi)};
}

__device__ __forceinline__ int pml_plane_a(int k, int nz, int npml) {
  if (k < npml) return k;
  if (k >= nz - npml) return npml + (k - (nz - npml));
  return -1;
}

template <typename T>
__device__ __forceinline__ const T* prof_a(const FdArgs& a, size_t off_d, size_t off_f) {
  if constexpr (sizeof(T) == 8)
    return reinterpret_cast<const T*>(a.ws + off_d);
  else
    return reinterpret_cast<const T*>(a.ws + off_f);
}

// E update, first half: with lambda' after the update, form lambda before it
// for E, J_D and the CPML auxiliaries, and the adjoints of the six H
// differences (scratch b_zy, b_zx, b_yz, b_xz, b_yx, b_xy).
template <typename T>
__global__ __launch_bounds__(256) void yee_e_adj_k1(FdAdjArgs aa) {
  const FdArgs& a = aa.f;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long n = static_cast<long>(nx) * ny * nz;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int k = static_cast<int>(idx / (static_cast<long>(nx) * ny));
  AdjPtr<T> f = adj_ptrs<T>(a);
  T* sc = static_cast<T*>(aa.scratch);
  T* E[3] = {f.Ex, f.Ey, f.Ez};
  T* JD[3] = {f.JDx, f.JDy, f.JDz};
  // every load of the cell before its first store: the arrays are distinct,
  // and with the stores in between each load would wait on the one before
  int m[3];
  T le[3], jd[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    m[c] = a.mat[c * n + idx];
    le[c] = E[c][idx];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) jd[c] = (m[c] == a.metal_id) ? JD[c][idx] : T(0);
  const int kk = pml_plane_a(k, nz, a.npml);
  const long plane = static_cast<long>(nx) * ny;
  const long np = 2L * a.npml * plane;
  const long o = kk * plane + (idx - static_cast<long>(k) * plane);
  T* psiEx = f.psi;
  T* psiEy = f.psi + np;
  T pex = T(0), pey = T(0);
  if (kk >= 0) {
    pex = psiEx[o];
    pey = psiEy[o];
  }
  T lcurl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c < 2 && k == 0) le[c] = T(0);  // those components are held at zero
    const T ce = static_cast<T>(a.ce[m[c] & 3]);
    lcurl[c] = ce * le[c];
    T lE = le[c];
    if (m[c] == a.metal_id) {
      const T ljd = jd[c] - ce * le[c];
      JD[c][idx] = static_cast<T>(a.alpha_d) * ljd;
      lE += static_cast<T>(a.beta_d) * ljd;
    }
    E[c][idx] = lE;
  }
  // curl_x = dHz_dy - dHy_dz~, curl_y = dHx_dz~ - dHz_dx, curl_z = dHy_dx - dHx_dy
  T b_zy = lcurl[0], b_yz = -lcurl[0], b_xz = lcurl[1], b_zx = -lcurl[1];
  const T b_yx = lcurl[2], b_xy = -lcurl[2];
  if (kk >= 0) {
    const T b = prof_a<T>(a, a.lay.bE, a.lay.bEf)[k];
    const T c = prof_a<T>(a, a.lay.aE, a.lay.aEf)[k];
    const T ki = prof_a<T>(a, a.lay.kE, a.lay.kEf)[k];
    const T tx = pex + b_yz;   // adjoint of psi_Ex' (total)
    const T ty = pey + b_xz;
    psiEx[o] = b * tx;
    psiEy[o] = b * ty;
    // ki b + c t with the fused product stated: left to the compiler, which
    // of the two it fuses follows the order of the code around it
    b_yz = fma_t(c, tx, ki * b_yz);
    b_xz = fma_t(ki, b_xz, c * ty);
  }
  sc[0 * n + idx] = b_zy;
  sc[1 * n + idx] = b_zx;
  sc[2 * n + idx] = b_yz;
  sc[3 * n + idx] = b_xz;
  sc[4 * n + idx] = b_yx;
  sc[5 * n + idx] = b_xy;
}

// E update, second half: lambda_H += curl^T of the difference adjoints.
template <typename T>
__global__ __launch_bounds__(256) void yee_e_adj_k2(FdAdjArgs aa) {
  const FdArgs& a = aa.f;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long n = static_cast<long>(nx) * ny * nz;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = static_cast<int>(idx % nx);
  const long jk = idx / nx;
  const int j = static_cast<int>(jk % ny);
  const int k = static_cast<int>(jk / ny);
  const long sy = nx, sz = static_cast<long>(nx) * ny;
  const long ip = (i + 1 == nx) ? idx - (nx - 1) : idx + 1;
  const long jp = (j + 1 == ny) ? idx - static_cast<long>(ny - 1) * sy : idx + sy;
  AdjPtr<T> f = adj_ptrs<T>(a);
  const T* sc = static_cast<const T*>(aa.scratch);
  const T inv_dx = static_cast<T>(a.inv_dx);
  const T* b_zy = sc;
  const T* b_zx = sc + n;
  const T* b_yz = sc + 2 * n;
  const T* b_xz = sc + 3 * n;
  const T* b_yx = sc + 4 * n;
  const T* b_xy = sc + 5 * n;
  // every load before the first store (see yee_e_adj_k1)
  const T hz = f.Hz[idx], hy = f.Hy[idx], hx = f.Hx[idx];
  // dHz_dy(c) = Hz[c] - Hz[c - y]; dHz_dx(c) = Hz[c] - Hz[c - x]
  const T dz = (b_zy[idx] - b_zy[jp] + b_zx[idx] - b_zx[ip]) * inv_dx;
  // dHy_dz(c) = Hy[c] - Hy[c - z] (Hy below k = 0 is zero); dHy_dx(c) = Hy[c] - Hy[c - x]
  const T yz_up = (k + 1 < nz) ? b_yz[idx + sz] : T(0);
  const T dy = (b_yz[idx] - yz_up + b_yx[idx] - b_yx[ip]) * inv_dx;
  const T xz_up = (k + 1 < nz) ? b_xz[idx + sz] : T(0);
  const T dx = (b_xz[idx] - xz_up + b_xy[idx] - b_xy[jp]) * inv_dx;
  f.Hz[idx] = hz + dz;
  f.Hy[idx] = hy + dy;
  f.Hx[idx] = hx + dx;
}

template <typename T>
__device__ __forceinline__ void gather_adj_cell(const CplAdjArgs& a, int c);

// H update, first half: difference adjoints a_* and the CPML auxiliaries.
// The blocks from cell_blocks on take the gather's adjoint, one occupied
// cell per thread: it adds to lambda_Ex, which this half neither reads nor
// writes, and the second half adds to lambda_E after it as before.
template <typename T>
__global__ __launch_bounds__(256) void yee_h_adj_k1(FdAdjArgs aa, CplAdjArgs gat, int cell_blocks) {
  if (static_cast<int>(blockIdx.x) >= cell_blocks) {
    const int c = (static_cast<int>(blockIdx.x) - cell_blocks) * 256 + static_cast<int>(threadIdx.x);
    if (c < gat.n_occ) gather_adj_cell<T>(gat, c);
    return;
  }
  const FdArgs& a = aa.f;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long n = static_cast<long>(nx) * ny * nz;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int k = static_cast<int>(idx / (static_cast<long>(nx) * ny));
  AdjPtr<T> f = adj_ptrs<T>(a);
  T* sc = static_cast<T*>(aa.scratch);
  const T cH = static_cast<T>(a.cH);
  const T lhx = f.Hx[idx], lhy = f.Hy[idx], lhz = f.Hz[idx];
  // Hx' = Hx - cH (dEz_dy - dEy_dz~); Hy' = Hy - cH (dEx_dz~ - dEz_dx);
  // Hz' = Hz - cH (dEy_dx - dEx_dy)
  const T a_zy = -cH * lhx;
  T a_yz = cH * lhx;
  T a_xz = -cH * lhy;
  const T a_zx = cH * lhy;
  const T a_yx = -cH * lhz;
  const T a_xy = cH * lhz;
  const int kk = pml_plane_a(k, nz, a.npml);
  if (kk >= 0) {
    const T b = prof_a<T>(a, a.lay.bH, a.lay.bHf)[k];
    const T c = prof_a<T>(a, a.lay.aH, a.lay.aHf)[k];
    const T ki = prof_a<T>(a, a.lay.kH, a.lay.kHf)[k];
    const long plane = static_cast<long>(nx) * ny;
    const long np = 2L * a.npml * plane;
    const long o = kk * plane + (idx - static_cast<long>(k) * plane);
    T* psiHx = f.psi + 2 * np;
    T* psiHy = f.psi + 3 * np;
    const T tx = psiHx[o] + a_yz;
    const T ty = psiHy[o] + a_xz;
    psiHx[o] = b * tx;
    psiHy[o] = b * ty;
    a_yz = ki * a_yz + c * tx;
    a_xz = ki * a_xz + c * ty;
  }
  sc[0 * n + idx] = a_zy;
  sc[1 * n + idx] = a_zx;
  sc[2 * n + idx] = a_yz;
  sc[3 * n + idx] = a_xz;
  sc[4 * n + idx] = a_yx;
  sc[5 * n + idx] = a_xy;
}

// H update, second half: lambda_E += curl^T of the difference adjoints.
template <typename T>
__global__ __launch_bounds__(256) void yee_h_adj_k2(FdAdjArgs aa) {
  const FdArgs& a = aa.f;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long n = static_cast<long>(nx) * ny * nz;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int i = static_cast<int>(idx % nx);
  const long jk = idx / nx;
  const int j = static_cast<int>(jk % ny);
  const int k = static_cast<int>(jk / ny);
  const long sy = nx, sz = static_cast<long>(nx) * ny;
  const long im = (i == 0) ? idx + (nx - 1) : idx - 1;
  const long jm = (j == 0) ? idx + static_cast<long>(ny - 1) * sy : idx - sy;
  AdjPtr<T> f = adj_ptrs<T>(a);
  const T* sc = static_cast<const T*>(aa.scratch);
  const T inv_dx = static_cast<T>(a.inv_dx);
  const T* a_zy = sc;
  const T* a_zx = sc + n;
  const T* a_yz = sc + 2 * n;
  const T* a_xz = sc + 3 * n;
  const T* a_yx = sc + 4 * n;
  const T* a_xy = sc + 5 * n;
  // every load before the first store (see yee_e_adj_k1)
  const T ez = f.Ez[idx], ey = f.Ey[idx], ex = f.Ex[idx];
  // dEz_dy(c) = Ez[c + y] - Ez[c]; dEz_dx(c) = Ez[c + x] - Ez[c]
  const T dz = (a_zy[jm] - a_zy[idx] + a_zx[im] - a_zx[idx]) * inv_dx;
  // dEy_dz(c) = Ey[c + z] - Ey[c] (Ey above the top is zero); dEy_dx(c) = Ey[c + x] - Ey[c]
  const T yz_dn = (k > 0) ? a_yz[idx - sz] : T(0);
  const T dy = (yz_dn - a_yz[idx] + a_yx[im] - a_yx[idx]) * inv_dx;
  const T xz_dn = (k > 0) ? a_xz[idx - sz] : T(0);
  const T dx = (xz_dn - a_xz[idx] + a_xy[jm] - a_xy[idx]) * inv_dx;
  f.Ez[idx] = ez + dz;
  f.Ey[idx] = ey + dy;
  f.Ex[idx] = ex + dx;
}

int launch_yee_e_adj(const FdAdjArgs& a, bool f32, hipStream_t s) {
  const long n = static_cast<long>(a.f.nx) * a.f.ny * a.f.nz;
  const int blocks = static_cast<int>((n + 255) / 256);
  if (f32) {
    hipLaunchKernelGGL(yee_e_adj_k1<float>, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(yee_e_adj_k2<float>, dim3(blocks), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(yee_e_adj_k1<double>, dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(yee_e_adj_k2<double>, dim3(blocks), dim3(256), 0, s, a);
  }
  return static_cast<int>(hipGetLastError());
}

int launch_yee_h_adj(const FdAdjArgs& a, const CplAdjArgs& gat, bool f32, hipStream_t s) {
  const long n = static_cast<long>(a.f.nx) * a.f.ny * a.f.nz;
  const int blocks = static_cast<int>((n + 255) / 256);
  const int gblocks = gat.n_occ > 0 ? (gat.n_occ + 255) / 256 : 0;
  if (f32) {
    hipLaunchKernelGGL(yee_h_adj_k1<float>, dim3(blocks + gblocks), dim3(256), 0, s, a, gat, blocks);
    hipLaunchKernelGGL(yee_h_adj_k2<float>, dim3(blocks), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(yee_h_adj_k1<double>, dim3(blocks + gblocks), dim3(256), 0, s, a, gat, blocks);
    hipLaunchKernelGGL(yee_h_adj_k2<double>, dim3(blocks), dim3(256), 0, s, a);
  }
  return static_cast<int>(hipGetLastError());
}

// g = coef sum over the source plane of ce[mat] lambda_Ex: one workgroup of
// 1024 threads, each summing a strided share of the plane in a fixed order,
// then a fixed tree (the plane is a few tens of thousands of cells).
constexpr int kSrcGradThreads = 1024;

template <typename T>
__device__ __forceinline__ void src_grad_block(const FdArgs& a, double coef, double* g_out) {
  __shared__ double red[kSrcGradThreads];
  const long plane = static_cast<long>(a.nx) * a.ny;
  const long o = static_cast<long>(a.src_k) * plane;
  const T* lEx = static_cast<const T*>(a.Ex);
  const double c0 = a.ce[0], c1 = a.ce[1], c2 = a.ce[2], c3 = a.ce[3];
  double s = 0.0;
  for (long p = threadIdx.x; p < plane; p += kSrcGradThreads) {
    const int m = a.mat[o + p] & 3;
    const double lo = (m & 1) ? c1 : c0, hi = (m & 1) ? c3 : c2;
    s += ((m & 2) ? hi : lo) * static_cast<double>(lEx[o + p]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSrcGradThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) g_out[0] = coef * red[0];
}

// -------------------------------------------------------------- coupling
// Forward: E_x[cell] -= ce (P' - P)/dt with P' = pfac sum_i d_i.
template <typename T>
__device__ __forceinline__ void deposit_adj_cell(const CplAdjArgs& a, int c) {
  const int cell = a.occ_cell[c];
  const double ce = a.ce[a.mat[cell] & 3];
  const double lex = static_cast<double>(static_cast<const T*>(a.lEx)[cell]);
  double lp_new;
  if (a.lJ == nullptr) {
    // one molecular step per field step: J = (P_new - P_old) / dt
    lp_new = a.lP[c] - ce * a.inv_dt * lex;
    a.lP[c] = ce * a.inv_dt * lex;
  } else {
    // multi-rate: E_x -= ce J at every step with J held between updates, so
    // the current's adjoint accumulates -ce lambda_Ex over the held steps;
    // at the update J = (P_new - P_old) / (M dt) hands it to both P's, and
    // the current before the update has no further influence
    const double lj = a.lJ[c] - ce * lex;
    if (!a.update) {
      a.lJ[c] = lj;
      return;
    }
    lp_new = a.lP[c] + a.inv_mdt * lj;
    a.lP[c] = -a.inv_mdt * lj;
    a.lJ[c] = 0.0;
  }
  const double ldv = a.pfac * lp_new;
  for (int t = a.occ_ptr[c]; t < a.occ_ptr[c + 1]; ++t) a.ld[a.mol_perm[t]] = ldv;
}

// Forward: E_mol,i = E_x[cell(i)] / E_au.
template <typename T>
__device__ __forceinline__ void gather_adj_cell(const CplAdjArgs& a, int c) {
  double s = 0.0;
  for (int t = a.occ_ptr[c]; t < a.occ_ptr[c + 1]; ++t) s += a.lE[a.mol_perm[t]];
  T* lEx = static_cast<T*>(a.lEx);
  const int cell = a.occ_cell[c];
  lEx[cell] = lEx[cell] + static_cast<T>(s * a.inv_eau);
}

// Block 0 forms the source gradient, the blocks after it take the deposit's
// adjoint, one occupied cell per thread: both read lambda_Ex as the E
// update's adjoint left it and write disjoint outputs.
template <typename T>
__global__ __launch_bounds__(kSrcGradThreads) void src_grad_deposit_adj_kernel(FdArgs f, double coef, double* g_out,
                                                                             CplAdjArgs dep) {
  if (blockIdx.x == 0) {
    src_grad_block<T>(f, coef, g_out);
    return;
  }
  const int c = (static_cast<int>(blockIdx.x) - 1) * kSrcGradThreads + static_cast<int>(threadIdx.x);
  if (c < dep.n_occ) deposit_adj_cell<T>(dep, c);
}

int launch_src_grad_deposit_adj(const FdArgs& lam, double coef, double* g_out, const CplAdjArgs& dep, bool f32,
                                hipStream_t s) {
  const int blocks = 1 + (dep.n_occ > 0 ? (dep.n_occ + kSrcGradThreads - 1) / kSrcGradThreads : 0);
  if (f32)
    hipLaunchKernelGGL(src_grad_deposit_adj_kernel<float>, dim3(blocks), dim3(kSrcGradThreads), 0, s, lam, coef,
                       g_out, dep);
  else
    hipLaunchKernelGGL(src_grad_deposit_adj_kernel<double>, dim3(blocks), dim3(kSrcGradThreads), 0, s, lam, coef,
                       g_out, dep);
  return static_cast<int>(hipGetLastError());
}

// ------------------------------------------------------------- objective
template <typename T>
__global__ __launch_bounds__(256) void yield_adj_init_kernel(cx<T>* lpsi, double* labs, const cx<T>* psi,
                                                             int n_mol, int lines, int n_r, int kdiss,
                                                             double dr, double scale) {
  const size_t per = static_cast<size_t>(lines) * n_r;
  const size_t total = per * n_mol;
  const T f = static_cast<T>(2.0 * dr * scale);
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int r = static_cast<int>(t % n_r);
    lpsi[t] = (r >= kdiss) ? cscale(psi[t], f) : cx<T>{T(0), T(0)};
    if (t % per == 0) labs[t / per] = scale;
  }
}

int launch_yield_adj_init(void* lpsi, double* labs, const void* psi, int n_mol, int lines, int n_r,
                          int kdiss, double dr, double scale, bool f32, hipStream_t s) {
  const size_t total = static_cast<size_t>(lines) * n_r * n_mol;
  size_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return 0;
  if (f32)
    hipLaunchKernelGGL(yield_adj_init_kernel<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<cx<float>*>(lpsi), labs, static_cast<const cx<float>*>(psi), n_mol,
                       lines, n_r, kdiss, dr, scale);
  else
    hipLaunchKernelGGL(yield_adj_init_kernel<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<cx<double>*>(lpsi), labs, static_cast<const cx<double>*>(psi), n_mol,
                       lines, n_r, kdiss, dr, scale);
  return static_cast<int>(hipGetLastError());
}

}  // namespace msqd
