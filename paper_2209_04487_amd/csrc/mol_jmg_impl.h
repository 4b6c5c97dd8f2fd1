// The molecular step in the rotational basis |j, m>, 2 <= j_max <= 5, with
// all three field components: one workgroup per molecule, (j_max + 1)^2
// lines per electronic state.  The coupling is the exact exponential on the
// truncated basis, applied as a rotation to the field frame, per-m' Gauss
// transforms of cos(theta), the 2x2 rotation of every eigenvector's (g, e)
// pair, and the way back (the construction and the tables are described in
// mol_jmg.h).
//
// Work decomposition: the line layout and the kinetic half-steps are those
// of the m = 0 step (R2 lanes per line, R1 values per lane, in-wave
// four-step FFT).  The lines go through LDS in SP rounds of radial points;
// in each round the coupling runs as three stages over the LDS rows:
//   A: per (state, j, r): y_m' = sum_m d^j_{m m'}(beta) e^{i m alpha} psi_m,
//   B: per (m', r): chi = Q^T y for both states, the increment of the
//      rotation, back with Q (the increments replace y in LDS),
//   C: per (state, j, r): dpsi_m = e^{-i m alpha} sum_m' d^j_{m m'} dy_m',
// and every lane adds the increments to the values it kept in registers
// (the increment form: rounding errors scale with the change, not with psi).
#pragma once

#include "mol_impl.h"
#include "mol_jmg.h"

namespace msqd {

// LDS of the per-molecule coupling tables: the phases e^{i m alpha}; d^j(beta)
// twice (row-major and transposed, rows padded to 16 bytes); Q and the
// scaled nodes; and the workgroup reduction scratch.
template <typename T, int JM>
struct JmgTabShape {
  static constexpr size_t a16(size_t b) { return (b + 15) / 16 * 16; }
  static constexpr JmgTab tab = jmg_tab(JM);
  static constexpr int PADE = 16 / static_cast<int>(sizeof(T));
  static constexpr int prow(int j) { return (2 * j + 1 + PADE - 1) / PADE * PADE; }
  static constexpr int poff(int j) { return j == 0 ? 0 : poff(j - 1) + (2 * j - 1) * prow(j - 1); }
  static constexpr int n_pad = poff(JM + 1);
  static constexpr size_t ph_bytes = a16(sizeof(cx<T>) * (2 * JM + 1));
  static constexpr size_t mt_bytes = a16(sizeof(T) * static_cast<size_t>(2 * n_pad + tab.n_q + tab.n_x));
  static constexpr size_t red_bytes = 6 * 16 * sizeof(double);
  static constexpr size_t bytes = ph_bytes + mt_bytes + red_bytes;
};

// Radial rounds of the line exchange.  Complex64 workgroups for j_max >= 4
// hold one molecule per CU whatever their LDS (their registers exclude a
// second), so they exchange all radial points in one round when the LDS
// allows it: half the barriers per step and twice the tasks per stage.  The
// others use the rounds of the m = 0 step, which keep the LDS of a
// workgroup small enough for several per CU.
template <typename T, int NR, int JM>
struct JmgSplit {
  static constexpr int R2 = FftShape<NR, T>::R2, L = 2 * (JM + 1) * (JM + 1);
  static constexpr size_t one_round = StagedTables<NR, T, true, false>::bytes +
                                      JmgTabShape<T, JM>::a16(sizeof(cx<T>) * static_cast<size_t>(lds_line_start(
                                                                                   L, NR + R2, sizeof(cx<T>)))) +
                                      JmgTabShape<T, JM>::bytes;
  static constexpr int value = (sizeof(T) == 4 && JM >= 4 && one_round <= 160 * 1024) ? 1 : fwd_split<NR, T>();
};

template <typename T, int NR, int JM>
struct JmgShape : JmgTabShape<T, JM> {
  typedef JmgTabShape<T, JM> TS;
  static constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2;
  static constexpr int NB = (JM + 1) * (JM + 1), L = 2 * NB, threads = L * R2;
  static constexpr int SP = JmgSplit<T, NR, JM>::value, NRH = NR / SP;
  static constexpr int LS = NRH + R2;   // line stride (elements) of the LDS rows
  typedef StagedTables<NR, T, true, false> TBL;
  static constexpr size_t rows_bytes =
      TS::a16(sizeof(cx<T>) * static_cast<size_t>(lds_line_start(L, LS, sizeof(cx<T>))));
  static constexpr size_t bytes = TBL::bytes + rows_bytes + TS::bytes;
  static constexpr bool fits = threads <= 1024 && bytes <= 160 * 1024;
};

// Start (elements) of line `line` in the LDS rows.
template <typename T, int NR, int JM>
__device__ __forceinline__ int jmg_row(int line) {
  return lds_line_start(line, JmgShape<T, NR, JM>::LS, static_cast<int>(sizeof(cx<T>)));
}

// ---------------------------------------------------------------- stages
// Task t of pass p for thread tid: the passes alternate direction, so that
// with tasks ordered from the heaviest down, a thread that drew a heavy task
// in one pass draws a light one in the next.  Only for workgroups of whole
// wavefronts: otherwise the reversed passes would split the tasks of one
// block over two wavefronts.
template <int NTHR>
__device__ __forceinline__ int zigzag_task(int pass, int tid) {
  return pass * NTHR + ((NTHR % 64 == 0 && (pass & 1)) ? NTHR - 1 - tid : tid);
}

// Workgroups of more than four whole wavefronts (nine at j_max = 5) put more
// of them on some SIMDs than on others, and with a fixed share of the tasks
// per wavefront those SIMDs set the pace of every stage.  Their stages
// therefore hand out the tasks dynamically: each wavefront takes the next 64
// (heaviest first) from an LDS counter, so the wavefronts that share a SIMD
// take fewer.  Every task writes only its own outputs, so the results do not
// depend on which wavefront takes it.
template <int NTHR>
inline constexpr bool kDynStages = NTHR % 64 == 0 && NTHR > 4 * 64;

// Run body(t) for t in [0, nt): dynamically (ctr: an LDS counter that is zero
// on entry) or in the zigzag passes.
template <int NTHR, typename F>
__device__ __forceinline__ void stage_tasks(int* ctr, int nt, int tid, F&& body) {
  if constexpr (kDynStages<NTHR>) {
    const int lane = tid & 63;
    for (;;) {
      int c = 0;
      if (lane == 0) c = atomicAdd(ctr, 1);
      c = __builtin_amdgcn_readfirstlane(c);
      if (c * 64 >= nt) break;
      const int t = c * 64 + lane;
      if (t < nt) body(t);
    }
  } else {
    for (int pass = 0; pass * NTHR < nt; ++pass) {
      const int t = zigzag_task<NTHR>(pass, tid);
      if (t < nt) body(t);
    }
  }
}

// Rotation of the j block of state s at radial point rl: to the field frame
// (BACK = false) or back (BACK = true).  dmr holds d^j(beta) row-major
// [m + j][m' + j] and dmt its transpose, each row padded to 16 bytes at
// JmgShape::poff(j), so that a row is read with 16-byte loads;
// ph[m + JM] = e^{i m alpha}.
template <typename T>
__device__ __forceinline__ void load_row16(T* dst, const T* src, int n) {
  if constexpr (sizeof(T) == 4) {
    for (int c = 0; c < n; c += 4) {
      const float4 w = *reinterpret_cast<const float4*>(src + c);
      dst[c] = w.x;
      dst[c + 1] = w.y;
      dst[c + 2] = w.z;
      dst[c + 3] = w.w;
    }
  } else {
    for (int c = 0; c < n; c += 2) {
      const double2 w = *reinterpret_cast<const double2*>(src + c);
      dst[c] = w.x;
      dst[c + 1] = w.y;
    }
  }
}

template <typename T, int NR, int JM, int J, bool BACK>
__device__ __forceinline__ void jmg_rot_block(cx<T>* sh, const T* dmr, const T* dmt, const cx<T>* ph, int s,
                                              int rl) {
  typedef JmgShape<T, NR, JM> S;
  constexpr int N = 2 * J + 1, NB = (JM + 1) * (JM + 1), P = S::prow(J);
  const T* d = (BACK ? dmr : dmt) + S::poff(J);
  cx<T>* row0 = sh + rl;
  const int l0 = s * NB + J * J;
  // the inputs stay in registers; each output goes to LDS as it is formed
  // (in place: the inputs were read before the first store)
  cx<T> u[N];
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = row0[jmg_row<T, NR, JM>(l0 + i)];
  if constexpr (!BACK) {
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = cmul(ph[JM - J + i], u[i]);
  }
#pragma unroll 1
  for (int o = 0; o < N; ++o) {
    // y_o = sum_i d[i][o] u_i (to the field frame, row o of the transpose)
    // or sum_i d[o][i] u_i (back, row o)
    T dv[P];
#pragma unroll
    for (int c = 0; c < P; c += S::PADE) load_row16(dv + c, d + o * P + c, S::PADE);
    cx<T> acc = cscale(u[0], dv[0]);
#pragma unroll
    for (int i = 1; i < N; ++i) acc = acc + cscale(u[i], dv[i]);
    if constexpr (BACK) acc = cmul_conj(acc, ph[JM - J + o]);
    row0[jmg_row<T, NR, JM>(l0 + o)] = acc;
  }
}

template <typename T, int NR, int JM, int J, bool BACK>
__device__ __forceinline__ void jmg_rot_dispatch(int j, cx<T>* sh, const T* dmr, const T* dmt, const cx<T>* ph,
                                                 int s, int rl) {
  if (j == J)
    jmg_rot_block<T, NR, JM, J, BACK>(sh, dmr, dmt, ph, s, rl);
  else if constexpr (J > 1)
    jmg_rot_dispatch<T, NR, JM, J - 1, BACK>(j, sh, dmr, dmt, ph, s, rl);
}

// All (state, j >= 1, r) tasks of a round; the j = 0 block is unchanged by
// the rotation.  Tasks are ordered by decreasing j so that the heavy blocks
// spread over the workgroup.
template <typename T, int NR, int JM, bool BACK>
__device__ __forceinline__ void jmg_rotate(cx<T>* sh, const T* dmr, const T* dmt, const cx<T>* ph, int tid,
                                           int* ctr) {
  constexpr int NRH = JmgShape<T, NR, JM>::NRH;
  constexpr int NT = 2 * JM * NRH;
  stage_tasks<JmgShape<T, NR, JM>::threads>(ctr, NT, tid, [&](int t) {
    const int jr = t / (2 * NRH);
    const int rem = t - jr * 2 * NRH;
    const int s = rem / NRH;
    jmg_rot_dispatch<T, NR, JM, JM, BACK>(JM - jr, sh, dmr, dmt, ph, s, rem - s * NRH);
  });
}

// Stage B on the block m' (|m'| = A) at radial point rl: the states
// j = A..JM of both electronic states.  The block |m'| = JM has the single
// state j = JM, on which cos(theta) vanishes: its increment is zero.
template <typename T, int NR, int JM, int A>
__device__ __forceinline__ void jmg_couple_block(cx<T>* sh, const T* qm, const T* xe, int mp, T md, int rl) {
  constexpr int N = JM + 1 - A, NB = (JM + 1) * (JM + 1);
  if constexpr (A == JM) {
    const int b = JM * JM + mp + JM;
    sh[jmg_row<T, NR, JM>(b) + rl] = {T(0), T(0)};
    sh[jmg_row<T, NR, JM>(NB + b) + rl] = {T(0), T(0)};
  } else {
    // Two passes, so that inputs and outputs are never live together.
    // (1) per eigenvector k: chi_k = sum_i Q[i][k] y_i for both states and
    //     its rotation increment dchi_k, stored at once over the block's LDS
    //     slots (all inputs are in registers by then; qm holds Q
    //     column-major, so column k is contiguous);
    // (2) per row i: dy_i = sum_k Q[i][k] dchi_k, read back from those slots.
    const T* Qc = qm + jmg_q_off(JM, A);
    const T* x = xe + jmg_x_off(JM, A);
    // the rotation angles' sine and versine first, while little else is
    // live (the large-angle path is an out-of-line call)
    T sn[N], vs[N];
#pragma unroll
    for (int k = 0; k < N; ++k) sin_vers(md * x[k], &sn[k], &vs[k]);
    cx<T> g[N], e[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int j = A + i, b = j * j + mp + j;
      g[i] = sh[jmg_row<T, NR, JM>(b) + rl];
      e[i] = sh[jmg_row<T, NR, JM>(NB + b) + rl];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const T* qk = Qc + k * N;
      cx<T> ag = cscale(g[0], qk[0]), ae = cscale(e[0], qk[0]);
#pragma unroll
      for (int i = 1; i < N; ++i) {
        ag = ag + cscale(g[i], qk[i]);
        ae = ae + cscale(e[i], qk[i]);
      }
      // exp(i th sigma_x) - 1 on (g, e): (-vers g + i sin e, i sin g - vers e)
      const int j = A + k, b = j * j + mp + j;   // slot k of the block
      sh[jmg_row<T, NR, JM>(b) + rl] = {-vs[k] * ag.x - sn[k] * ae.y, -vs[k] * ag.y + sn[k] * ae.x};
      sh[jmg_row<T, NR, JM>(NB + b) + rl] = {-vs[k] * ae.x - sn[k] * ag.y, -vs[k] * ae.y + sn[k] * ag.x};
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int j = A + k, b = j * j + mp + j;
      g[k] = sh[jmg_row<T, NR, JM>(b) + rl];
      e[k] = sh[jmg_row<T, NR, JM>(NB + b) + rl];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      cx<T> ag = cscale(g[0], Qc[i]), ae = cscale(e[0], Qc[i]);
#pragma unroll
      for (int k = 1; k < N; ++k) {
        ag = ag + cscale(g[k], Qc[k * N + i]);
        ae = ae + cscale(e[k], Qc[k * N + i]);
      }
      const int j = A + i, b = j * j + mp + j;
      sh[jmg_row<T, NR, JM>(b) + rl] = ag;
      sh[jmg_row<T, NR, JM>(NB + b) + rl] = ae;
    }
  }
}

template <typename T, int NR, int JM, int A>
__device__ __forceinline__ void jmg_couple_dispatch(int a, cx<T>* sh, const T* qm, const T* xe, int mp, T md,
                                                    int rl) {
  if (a == A)
    jmg_couple_block<T, NR, JM, A>(sh, qm, xe, mp, md, rl);
  else if constexpr (A > 0)
    jmg_couple_dispatch<T, NR, JM, A - 1>(a, sh, qm, xe, mp, md, rl);
}

// All (m', r) tasks of a round, m' in the order 0, 1, -1, 2, -2, ...
template <typename T, int NR, int JM>
__device__ __forceinline__ void jmg_couple(cx<T>* sh, const T* qm, const T* xe, const T* mudt_h, int tid,
                                           int* ctr) {
  constexpr int NRH = JmgShape<T, NR, JM>::NRH;
  constexpr int NT = (2 * JM + 1) * NRH;
  stage_tasks<JmgShape<T, NR, JM>::threads>(ctr, NT, tid, [&](int t) {
    const int u = t / NRH;
    const int rl = t - u * NRH;
    const int a = (u + 1) >> 1;
    const int mp = (u & 1) ? a : -a;
    jmg_couple_dispatch<T, NR, JM, JM>(a, sh, qm, xe, mp, mudt_h[rl], rl);
  });
}

// The terms of the dipole vector at radial point rl from the basis states of
// one j (FP64): Re<g|D_z|e>, and P = <g|D_+|e>, P' = <e|D_+|g> with
// D_+ = D_x + i D_y, from which Re<g|D_x|e> = (Re P + Re P') / 2 and
// Re<g|D_y|e> = (Im P + Im P') / 2.  Summed over j they give the dipole.
template <typename T, int NR, int JM>
__device__ __forceinline__ void jmg_dipole_point(const cx<T>* sh, const double* dip, int j, int rl, double* tx,
                                                 double* ty, double* tz) {
  constexpr int NB = (JM + 1) * (JM + 1);
  auto ld = [&](int line) {
    const cx<T> v = sh[jmg_row<T, NR, JM>(line) + rl];
    return cx<double>{static_cast<double>(v.x), static_cast<double>(v.y)};
  };
  double z = 0.0, pr = 0.0, pi = 0.0;
#pragma unroll 1
  for (int m = -j; m <= j; ++m) {
    const int b = j * j + m + j;
    const cx<double> gb = ld(b), eb = ld(NB + b);
    if (j < JM) {
      const int bz = (j + 1) * (j + 1) + m + j + 1;        // (j+1, m)
      const int bp = bz + 1;                               // (j+1, m+1)
      const cx<double> gz = ld(bz), ez = ld(NB + bz);
      z += dip[3 * b] * ((gz.x * eb.x + gz.y * eb.y) + (gb.x * ez.x + gb.y * ez.y));
      const cx<double> gp = ld(bp), ep = ld(NB + bp);
      const double c = dip[3 * b + 1];
      // conj(g_p) e_b + conj(e_p) g_b
      pr += c * ((gp.x * eb.x + gp.y * eb.y) + (ep.x * gb.x + ep.y * gb.y));
      pi += c * ((gp.x * eb.y - gp.y * eb.x) + (ep.x * gb.y - ep.y * gb.x));
    }
    if (m + 1 <= j - 1) {
      const int bm = (j - 1) * (j - 1) + m + 1 + j - 1;    // (j-1, m+1)
      const cx<double> gm = ld(bm), em = ld(NB + bm);
      const double c = dip[3 * b + 2];
      pr += c * ((gm.x * eb.x + gm.y * eb.y) + (em.x * gb.x + em.y * gb.y));
      pi += c * ((gm.x * eb.y - gm.y * eb.x) + (em.x * gb.y - em.y * gb.x));
    }
  }
  *tx = 0.5 * pr;
  *ty = 0.5 * pi;
  *tz = z;
}

// ---------------------------------------------------------------- kernel
// Waves per SIMD the register allocation targets (complex64): three where
// that fits more workgroups on a CU than two does.  A seven-wave workgroup
// (j_max = 4 at R2 = 8) gets one workgroup per CU either way, so it keeps
// two waves per SIMD and the registers that come with them.
template <typename T, int NR, int JM>
struct JmgOcc {
  static constexpr int wg_waves = (JmgShape<T, NR, JM>::threads + 63) / 64;
  static constexpr int waves = sizeof(T) == 8 ? 1 : ((12 / wg_waves) > (8 / wg_waves) ? 3 : 2);
};

template <typename T, int NR, int JM, bool ONE>
__global__ __launch_bounds__((JmgShape<T, NR, JM>::threads)) __attribute__((amdgpu_waves_per_eu(JmgOcc<T, NR, JM>::waves)))
void mol_jmg_kernel(MolArgs a) {
  typedef JmgShape<T, NR, JM> S;
  constexpr int R1 = S::R1, R2 = S::R2, NB = S::NB, SP = S::SP, PH = R1 / SP, NRH = S::NRH;
  constexpr JmgTab TB = S::tab;
  typedef typename S::TBL TBL;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* kin_s = reinterpret_cast<cx<T>*>(smem);
  cx<T>* tw_s = kin_s + NR;
  T* mask_s = reinterpret_cast<T*>(tw_s + TBL::tw_elems);
  cx<T>* sh = reinterpret_cast<cx<T>*>(smem + TBL::bytes);
  cx<T>* ph = reinterpret_cast<cx<T>*>(smem + TBL::bytes + S::rows_bytes);
  T* dmr = reinterpret_cast<T*>(smem + TBL::bytes + S::rows_bytes + S::ph_bytes);
  T* dmt = dmr + S::n_pad;
  T* qm = dmt + S::n_pad;
  T* xe = qm + TB.n_q;
  double* red = reinterpret_cast<double*>(smem + TBL::bytes + S::rows_bytes + S::ph_bytes + S::mt_bytes);
  // the stages' task counters live in the reduction area, which is used
  // only after the last stage
  int* ctr = reinterpret_cast<int*>(red);

  const int mol = blockIdx.x;
  const int tid = threadIdx.x;
  constexpr int nthr = S::threads;
  const int line = tid / R2;
  const int q = tid - line * R2;
  const int st = line / NB, b = line - st * NB;
  int jl = 0;
  while ((jl + 1) * (jl + 1) <= b) ++jl;

  const char* ws = a.ws;
  const bool dbl = sizeof(T) == 8;
  const cx<T>* kin_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.kin_d : a.lay.kin_f));
  const cx<T>* tw_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.tw_d : a.lay.tw_f));
  const cx<T>* vph_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.vph_d : a.lay.vph_f));
  const T* mudt = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mudt_d : a.lay.mudt_f));
  const T* mask_g = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mask_d : a.lay.mask_f));
  const double* mu = reinterpret_cast<const double*>(ws + a.lay.mu_d);
  const double* tg = reinterpret_cast<const double*>(ws + a.lay.total);

  // field at the molecule (each component at its own edge of the cell);
  // a readout-only launch (no step) reads no field
  double E3[3] = {0.0, 0.0, 0.0};
  if (a.n_steps > 0) {
    if (a.Ex != nullptr) {
      const int c = a.cell_of_mol[mol];
      const void* f3[3] = {a.Ex, a.Ey, a.Ez};
#pragma unroll
      for (int k = 0; k < 3; ++k)
        E3[k] = (a.ex_is_float ? static_cast<double>(static_cast<const float*>(f3[k])[c])
                               : static_cast<const double*>(f3[k])[c]) * a.inv_eau;
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) E3[k] = a.E_mol[3 * mol + k];
    }
  }
  if (a.E_out != nullptr && tid == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.E_out[3 * mol + k] = E3[k];
  }

  cx<T>* psi = reinterpret_cast<cx<T>*>(a.psi) + static_cast<size_t>(mol) * S::L * NR;
  cx<T>* slot = sh + jmg_row<T, NR, JM>(line);
  const int loff = line * NR + q;
  const int voff = (st * a.nj + jl) * NR + q;   // potential phases depend on (state, j)
  cx<T> vv[R1];
#pragma unroll
  for (int p = 0; p < R1; ++p) vv[p] = psi[loff + R2 * p];

  // per-molecule coupling tables: the field frame (alpha, beta) and |E|
  {
    const double en = sqrt(E3[0] * E3[0] + E3[1] * E3[1] + E3[2] * E3[2]);
    const double rho = sqrt(E3[0] * E3[0] + E3[1] * E3[1]);
    const double ca = rho > 0.0 ? E3[0] / rho : 1.0, sa = rho > 0.0 ? E3[1] / rho : 0.0;
    const double cb = en > 0.0 ? E3[2] / en : 1.0, sb = en > 0.0 ? rho / en : 0.0;
    if (tid < 2 * JM + 1) {
      const int m = tid - JM, am = m < 0 ? -m : m;
      double px = 1.0, py = 0.0;
      for (int k = 0; k < am; ++k) {
        const double nx = px * ca - py * sa;
        py = px * sa + py * ca;
        px = nx;
      }
      ph[tid] = {static_cast<T>(px), static_cast<T>(m < 0 ? -py : py)};
    }
    // d^j_{m m'}(beta) = sum_k O_{m k} O_{m' k} cos(pi/2 (m' - m) - beta mu_k),
    // mu_k = k - j: ra, rc are the rows of m and m' in O
    auto wigner_d = [&](int j, int ra, int rc) {
      const int n = 2 * j + 1;
      const double* O = tg + TB.jx + jmg_jx_off(j);
      // cos(pi/2 (m' - m) - beta mu) = cA cos(mu beta) + sA sin(mu beta)
      const int dq = (rc - ra) & 3;
      const double cA = dq == 0 ? 1.0 : (dq == 2 ? -1.0 : 0.0);
      const double sA = dq == 1 ? 1.0 : (dq == 3 ? -1.0 : 0.0);
      double acc = O[ra * n + j] * O[rc * n + j] * cA;
      double wc = 1.0, wsn = 0.0;   // cos(mu beta), sin(mu beta)
      for (int mu_ = 1; mu_ <= j; ++mu_) {
        const double nc = wc * cb - wsn * sb;
        wsn = wc * sb + wsn * cb;
        wc = nc;
        acc += O[ra * n + j + mu_] * O[rc * n + j + mu_] * (cA * wc + sA * wsn) +
               O[ra * n + j - mu_] * O[rc * n + j - mu_] * (cA * wc - sA * wsn);
      }
      return acc;
    };
    // both padded layouts: entry (row r, column c) of block j is d[r][c]
    // in dmr and d[c][r] in dmt; the padding columns are zero
    for (int t = tid; t < S::n_pad; t += nthr) {
      int j = 0;
      while (t >= S::poff(j + 1)) ++j;
      const int P = S::prow(j), o = t - S::poff(j), r = o / P, c = o - r * P;
      const bool in = c < 2 * j + 1;
      dmr[t] = in ? static_cast<T>(wigner_d(j, r, c)) : T(0);
      dmt[t] = in ? static_cast<T>(wigner_d(j, c, r)) : T(0);
    }
    // Q^(a) column-major in LDS (the workspace holds it row-major)
    for (int t = tid; t < TB.n_q; t += nthr) {
      int am = 0;
      while (t >= jmg_q_off(JM, am + 1)) ++am;
      const int n = JM + 1 - am, o = t - jmg_q_off(JM, am), i = o / n, k = o - i * n;
      qm[jmg_q_off(JM, am) + k * n + i] = static_cast<T>(tg[TB.q + t]);
    }
    for (int t = tid; t < TB.n_x; t += nthr) xe[t] = static_cast<T>(en * tg[TB.x + t]);
  }
  if constexpr (stage_tables<NR, T>()) stage_tables_to_lds<NR, T, true>(kin_s, tw_s, mask_s, kin_g, tw_g, mask_g);
  __syncthreads();

  double ab = 0.0;
  const int n_steps = ONE ? 1 : a.n_steps;
  for (int step = 0; step < n_steps; ++step) {
    const cx<T>* kin;
    const cx<T>* tw;
    const T* mask;
    if constexpr (stage_tables<NR, T>()) {
      kin = kin_s;
      tw = tw_s;
      mask = mask_s;
    } else {
      kin = opaque(kin_g);
      tw = opaque(tw_g);
      mask = opaque(mask_g);
    }
    const cx<T>* vph = opaque(vph_g);
    kinetic_half<T, NR, false, SP, TBL::TWC>(vv, slot, q, kin, tw);
#pragma unroll
    for (int h = 0; h < SP; ++h) {
#pragma unroll
      for (int pp = 0; pp < PH; ++pp) {
        const int p = h * PH + pp;
        vv[p] = phase_mul(vv[p], vph[voff + R2 * p]);
        slot[q + R2 * pp] = vv[p];
      }
      // the previous round's stages ended at a barrier: reset their counters
      if (kDynStages<nthr> && tid == 0) ctr[0] = ctr[1] = ctr[2] = 0;
      __syncthreads();
      jmg_rotate<T, NR, JM, false>(sh, dmr, dmt, ph, tid, ctr);
      __syncthreads();
      jmg_couple<T, NR, JM>(sh, qm, xe, mudt + h * NRH, tid, ctr + 1);
      __syncthreads();
      jmg_rotate<T, NR, JM, true>(sh, dmr, dmt, ph, tid, ctr + 2);
      __syncthreads();
#pragma unroll
      for (int pp = 0; pp < PH; ++pp) {
        const int p = h * PH + pp;
        vv[p] = phase_mul(vv[p] + slot[q + R2 * pp], vph[voff + R2 * p]);
      }
    }
    kinetic_half<T, NR, false, SP, TBL::TWC>(vv, slot, q, kin, tw);
    constexpr int P0 = (3 * R1) / 4;
    if (a.kmask >= R2 * P0) {
#pragma unroll
      for (int p = P0; p < R1; ++p) absorb_point_nb(vv[p], mask[q + R2 * p], ab);
    } else {
#pragma unroll
      for (int p = 0; p < R1; ++p) absorb_point(vv[p], mask[q + R2 * p], ab);
    }
  }

  // readouts: norm, yield, and the dipole vector (in the same rounds)
  double nrm = 0.0, yld = 0.0;
#pragma unroll
  for (int p = 0; p < R1; ++p) {
    const double n2 = static_cast<double>(norm2(vv[p]));
    nrm += n2;
    if (q + R2 * p >= a.kdiss) yld += n2;
  }
  double dc[3] = {0.0, 0.0, 0.0};
  if (a.want_d && a.d_mol) {
    const double* dip = tg + TB.dip;
#pragma unroll
    for (int h = 0; h < SP; ++h) {
      __syncthreads();   // the previous users of the slots are done
#pragma unroll
      for (int pp = 0; pp < PH; ++pp) slot[q + R2 * pp] = vv[h * PH + pp];
      __syncthreads();
      for (int pass = 0; pass * nthr < NRH * (JM + 1); ++pass) {
        const int t = zigzag_task<JmgShape<T, NR, JM>::threads>(pass, tid);
        if (t >= NRH * (JM + 1)) continue;
        const int j = JM - t / NRH, rl = t - (JM - j) * NRH;   // heaviest j first
        double tx, ty, tz;
        jmg_dipole_point<T, NR, JM>(sh, dip, j, rl, &tx, &ty, &tz);
        const double m = mu[h * NRH + rl];
        dc[0] += m * tx;
        dc[1] += m * ty;
        dc[2] += m * tz;
      }
    }
  }
  // workgroup sums of (ab, nrm, yld, dx, dy, dz) in a fixed order
  double vals[6] = {ab, nrm, yld, dc[0], dc[1], dc[2]};
  const int lane = tid & 63, wid = tid >> 6;
  constexpr int nw = (nthr + 63) >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) vals[k] = wave_sum(vals[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wid * 6 + k] = vals[k];
  }
  __syncthreads();
  if (tid == 0) {
    double sm[6];
    for (int k = 0; k < 6; ++k) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w * 6 + k];
      sm[k] = t;
    }
    const double dr = a.dr;
    const double absorbed = a.absorbed[mol] + sm[0] * dr;
    if (n_steps > 0) a.absorbed[mol] = absorbed;
    if (a.want_d && a.d_mol) {
      for (int k = 0; k < 3; ++k) a.d_mol[3 * mol + k] = 2.0 * dr * sm[3 + k];
    }
    if (a.want_norm && a.norm_mol) a.norm_mol[mol] = sm[1] * dr;
    if (a.want_yield && a.yield_mol) a.yield_mol[mol] = sm[2] * dr + absorbed;
    if (!isfinite(sm[1]) || !isfinite(sm[3]) || !isfinite(sm[4]) || !isfinite(sm[5]) || !isfinite(absorbed))
      atomicOr(a.status, 1);
  }
  if (n_steps > 0) {
#pragma unroll
    for (int p = 0; p < R1; ++p) psi[loff + R2 * p] = vv[p];
  }
}

template <typename T, int NR, int JM, bool ONE>
int launch_jmg_t1(const MolArgs& a, hipStream_t s) {
  typedef JmgShape<T, NR, JM> S;
  if constexpr (!S::fits) {
    return static_cast<int>(hipErrorInvalidValue);
  } else {
    const size_t shm = S::bytes;
    if (shm > mol_lds_limit()) return static_cast<int>(hipErrorInvalidValue);
    static std::atomic<unsigned long long> lds_set{0};
    if (shm > 64 * 1024) {
      const hipError_t e = allow_large_lds(reinterpret_cast<const void*>(&mol_jmg_kernel<T, NR, JM, ONE>), lds_set);
      if (e != hipSuccess) return static_cast<int>(e);
    }
    hipLaunchKernelGGL((mol_jmg_kernel<T, NR, JM, ONE>), dim3(a.n_mol), dim3(S::threads), shm, s, a);
    return static_cast<int>(hipGetLastError());
  }
}

template <typename T, int NR, int JM>
int launch_jmg_t(const MolArgs& a, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (a.n_steps == 1) return launch_jmg_t1<T, NR, JM, true>(a, s);
  }
  return launch_jmg_t1<T, NR, JM, false>(a, s);
}

template <typename T, int JM>
int launch_jmg_nr(const MolArgs& a, int n_r, hipStream_t s) {
  switch (n_r) {
    case 64: return launch_jmg_t<T, 64, JM>(a, s);
    case 128: return launch_jmg_t<T, 128, JM>(a, s);
    case 256: return launch_jmg_t<T, 256, JM>(a, s);
    case 512: return launch_jmg_t<T, 512, JM>(a, s);
    default: return static_cast<int>(hipErrorInvalidValue);
  }
}

template <typename T>
int launch_jmg_prec(const MolArgs& a, int n_r, int jm, hipStream_t s) {
  switch (jm) {
    case 2: return launch_jmg_nr<T, 2>(a, n_r, s);
    case 3: return launch_jmg_nr<T, 3>(a, n_r, s);
    case 4: return launch_jmg_nr<T, 4>(a, n_r, s);
    case 5: return launch_jmg_nr<T, 5>(a, n_r, s);
    default: return static_cast<int>(hipErrorInvalidValue);
  }
}

template <typename T, int JM>
bool jmg_fits_nr(int n_r, size_t* lds) {
  switch (n_r) {
    case 64: *lds = JmgShape<T, 64, JM>::bytes; return JmgShape<T, 64, JM>::fits;
    case 128: *lds = JmgShape<T, 128, JM>::bytes; return JmgShape<T, 128, JM>::fits;
    case 256: *lds = JmgShape<T, 256, JM>::bytes; return JmgShape<T, 256, JM>::fits;
    case 512: *lds = JmgShape<T, 512, JM>::bytes; return JmgShape<T, 512, JM>::fits;
    default: *lds = 0; return false;
  }
}

template <typename T>
bool jmg_fits(int n_r, int jm, size_t* lds) {
  switch (jm) {
    case 2: return jmg_fits_nr<T, 2>(n_r, lds);
    case 3: return jmg_fits_nr<T, 3>(n_r, lds);
    case 4: return jmg_fits_nr<T, 4>(n_r, lds);
    case 5: return jmg_fits_nr<T, 5>(n_r, lds);
    default: *lds = 0; return false;
  }
}

}  // namespace msqd
