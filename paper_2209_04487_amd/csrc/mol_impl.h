// Fused molecular step for one molecule per workgroup.
//
// One split-operator step (K/2 V/2 C(E) V/2 K/2, absorber) of the two-state
// wavepacket of Eqs. (3)-(5), with the angular part of the coupling in Eq. (4)
// integrated on the Gauss-Legendre angular grid.  The whole molecule stays on
// chip for the step (and for every step of a multi-step call): psi crosses
// HBM once in each direction.
//
// Work decomposition inside the workgroup
//   line layout : line (s, J) is owned by R2 consecutive lanes; lane q holds
//                 r = q + R2 p, p = 0..R1-1 (n_r = R1 R2) in registers.
//                 K/2 = two in-register DFT passes with an LDS transpose in
//                 between (four-step FFT), kinetic phase, and the inverse.
//                 All exchanges of a line stay inside one wavefront.
//   r layout    : one lane per radial point holds all (s, J) of that point
//                 (read from the line slots in LDS): J <-> angle transform,
//                 per-node 2x2 rotation, readouts.
#pragma once

#include "fft_reg.h"
#include "host_tables.h"
#include "mol.h"

namespace msqd {

// n_r = R1 * R2: each lane holds R1 values of a line, R2 lanes per line.
// The split is the host's fft_r1(n_r, element bytes): complex64 lines use
// longer in-register DFTs (fewer lanes and waves per molecule, more
// molecules per CU); complex128 keeps R1 <= 16 within the register file.
template <int NR, typename T>
struct FftShape {
  static constexpr int R1 = fft_r1(NR, static_cast<int>(sizeof(T)));
  static constexpr int R2 = NR / R1;
};

template <int NR, typename T>
constexpr int line_stride() { return NR + FftShape<NR, T>::R2; }

// The fused forward step exchanges each line through LDS in SP rounds of
// NR/SP radial points (the in-line transposes and the J<->angle exchange
// alike), so that a molecule needs 1/SP of the LDS and more molecules fit on
// a CU.  complex64 lines with an even number of columns per lane use two
// rounds; complex128 lines (register-bound, one molecule per CU either way)
// and the shortest grids use one.
template <int NR, typename T>
constexpr int fwd_split() {
  return (sizeof(T) == 4 && (FftShape<NR, T>::R1 / FftShape<NR, T>::R2) % 2 == 0) ? 2 : 1;
}
template <int NR, typename T>
constexpr int fwd_line_stride() { return NR / fwd_split<NR, T>() + FftShape<NR, T>::R2; }

// The per-workgroup LDS copy of the transform tables (kinetic factors,
// four-step twiddles, absorber mask), kept ahead of the lines (complex64
// forms only: the complex128 form holds one molecule per CU, where the staged
// tables measured slower than reading them through the caches).  The twiddle
// table is either the full R1 x R1 table or, with COMPACT, only the R2 rows
// that the transforms read, in rows of R1 + 1 (the pad spreads the lanes of a
// line over distinct banks): the compact form is for kernels whose
// occupancy is bounded by LDS.
//
// With CPOPS the copy also holds the operands of the J <-> angle contraction
// (the matrix-core fragments of T and T^T, 2 KB, and the angle nodes padded
// with zeros to 16), which every exchange round of every step reads.
template <int NR, typename T, bool COMPACT = false, bool CPOPS = true>
struct StagedTables {
  static constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2;
  static constexpr bool on = sizeof(T) == 4;
  static constexpr int TWC = (on && COMPACT) ? R1 + 1 : 0;   // compact row stride (0: full layout)
  static constexpr size_t tw_elems =
      on ? (COMPACT ? static_cast<size_t>(R2) * (R1 + 1) : static_cast<size_t>(R1) * R1) : 0;
  static constexpr size_t fft_bytes = (NR * sizeof(cx<T>) + tw_elems * sizeof(cx<T>) + NR * sizeof(T) + 15) / 16 * 16;
  static constexpr size_t frag_bytes = 4 * 64 * 4 * 2;   // bf16 [4][64][4] or float [2][64][4]
  static constexpr int x_pad = 16;
  static constexpr size_t cp_bytes = (on && CPOPS) ? frag_bytes + x_pad * sizeof(float) : 0;
  static constexpr size_t bytes = on ? fft_bytes + cp_bytes : 0;
};
template <int NR, typename T>
constexpr bool stage_tables() { return StagedTables<NR, T>::on; }
template <int NR, typename T>
constexpr size_t lds_table_bytes() { return StagedTables<NR, T>::bytes; }

// Cooperative copy of a table into LDS in 16-byte pieces.
__device__ __forceinline__ void lds_stage(void* dst, const void* src, size_t bytes) {
  const uint4* s = static_cast<const uint4*>(src);
  uint4* d = static_cast<uint4*>(dst);
  for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// Stage the tables: kin [NR], the twiddles of the R1 x R1 table tw_g (all,
// or the rows x < R2 in the compact layout), and mask [NR]; the caller
// synchronises the workgroup afterwards.
template <int NR, typename T, bool COMPACT = false>
__device__ __forceinline__ void stage_tables_to_lds(cx<T>* kin_s, cx<T>* tw_s, T* mask_s, const cx<T>* kin_g,
                                                    const cx<T>* tw_g, const T* mask_g) {
  typedef StagedTables<NR, T, COMPACT, false> ST;
  lds_stage(kin_s, kin_g, NR * sizeof(cx<T>));
  if constexpr (COMPACT) {
    for (int t = threadIdx.x; t < ST::R2 * ST::R1; t += blockDim.x) tw_s[(t / ST::R1) * ST::TWC + t % ST::R1] = tw_g[t];
  } else {
    lds_stage(tw_s, tw_g, ST::tw_elems * sizeof(cx<T>));
  }
  lds_stage(mask_s, mask_g, NR * sizeof(T));
}

template <int NR, typename T>
__device__ __forceinline__ int lds_row(int line) {
  return lds_line_start(line, fwd_line_stride<NR, T>(), static_cast<int>(sizeof(cx<T>)));
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hide a uniform pointer's value from the optimiser so that table loads stay
// inside the step loop instead of being hoisted into (many) live registers.
// The barrier acts on a global-address-space copy of the pointer, so that
// loads through the result stay global loads (a generic pointer would turn
// them into flat loads, which also count against the LDS wait counter and
// make every LDS wait also wait for the table loads in flight).
template <typename P>
__device__ __forceinline__ P* opaque(P* p) {
  using GP = __attribute__((address_space(1))) P*;
  GP g = (GP)p;
  asm volatile("" : "+s"(g));
  return (P*)g;
}

template <typename T>
__device__ __forceinline__ cx<T> cmul_conj(cx<T> a, cx<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// Unit phase factors from the kinetic and potential tables: the FP64 tables
// hold (cos, sin), the FP32 tables the lifting parameters (-tan(phi/2),
// sin phi) of the same angle (see lift_rot).
template <typename T>
__device__ __forceinline__ cx<T> phase_mul(cx<T> v, cx<T> t) {
  if constexpr (sizeof(T) == 8)
    return cmul(v, t);
  else
    return lift_rot(v, t.x, t.y);
}
template <typename T>
__device__ __forceinline__ cx<T> phase_mul_conj(cx<T> v, cx<T> t) {
  if constexpr (sizeof(T) == 8)
    return cmul_conj(v, t);
  else
    return lift_rot(v, -t.x, -t.y);
}
// kinetic factor: the FP64 table carries the 1/NR of the inverse transform,
// the FP32 form applies it as an exact power-of-two scale after the rotation
template <typename T, int NR, bool CONJ>
__device__ __forceinline__ cx<T> kin_mul(cx<T> v, cx<T> t) {
  if constexpr (sizeof(T) == 8) {
    return CONJ ? cmul_conj(v, t) : cmul(v, t);
  } else {
    const cx<T> w = CONJ ? phase_mul_conj(v, t) : phase_mul(v, t);
    return cscale(w, T(1) / T(NR));
  }
}

template <typename T>
struct MolTabs {
  const cx<T>* kin;
  const cx<T>* tw;
  const cx<T>* vph;
  const T* x;
  const T* mudt;
  const T* mask;
  const double* mu;
  const double* cj;
};

// ---------------------------------------------------------------- K/2
// v: this lane's R1 values of its line (r = q + R2 p); slot: the line's LDS
// region (R2 * (R1 + 1) elements).  kin is applied by kin_mul, which
// includes the 1/NR of the inverse transform.  tw2[x * R1 + y] = exp(-2 pi i x y / NR) for
// x, y < R1, so that every table access is a uniform base plus one lane
// offset plus an immediate.  With TWC > 0 the table is the compact one that
// holds only the rows x < R2 that are read (exp(-2 pi i x y / NR) at
// x * TWC + y, TWC >= R1): one lane offset x = q serves both passes.
// With TWS (complex64, n_r an even power of two) the table holds the
// twiddles times n_r^(-1/2): each pass then scales by n_r^(-1/2) through its
// twiddles, and the first row and column, which have none, by an explicit
// power of two, so that the inverse transform's 1/n_r costs no multiply per
// element (the rounded results are those of the unscaled passes times
// exact powers of two).
template <int NR>
constexpr int tw_log2() { return NR <= 1 ? 0 : 1 + tw_log2<NR / 2>(); }
template <int NR, typename T>
constexpr bool tw_scaled() { return sizeof(T) == 4 && tw_log2<NR>() % 2 == 0; }

template <typename T, int NR, bool CONJ = false, int SP = 1, int TWC = 0, bool TWS = false>
__device__ __forceinline__ void kinetic_half(cx<T>* v, cx<T>* slot, int q, const cx<T>* __restrict__ kin,
                                             const cx<T>* __restrict__ tw2) {
  constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2, U = R1 / R2;
  // SP rounds of RH = R1/SP columns each; the slot holds R2 rows of RH + 1
  constexpr int RH = R1 / SP, UH = U / SP, RS = RH + 1;
  static_assert(U % SP == 0, "columns per lane must split evenly");
  static_assert(!TWS || tw_scaled<NR, T>(), "scaled twiddles need complex64 and an even log2 n_r");
  const T s_half = T(1) / T(1 << (tw_log2<NR>() / 2));   // n_r^(-1/2) (TWS)
  // pass 1: DFT over p, twiddle exp(-2 pi i q a / NR)
  dft<R1, false, T>(v);
  if constexpr (TWS) v[0] = cscale(v[0], s_half);
#pragma unroll
  for (int a = 1; a < R1; ++a) v[a] = cmul(v[a], TWC > 0 ? tw2[q * TWC + a] : tw2[a * R1 + q]);
#pragma unroll
  for (int h = 0; h < SP; ++h) {
    if (h > 0) wave_lds_sync();
    // this lane's row of the columns [h RH, (h+1) RH)
#pragma unroll
    for (int al = 0; al < RH; ++al) slot[q * RS + al] = v[h * RH + al];
    wave_lds_sync();
    // pass 2 on the transposed data: frequency k = a + R1 b, columns
    // a = q + R2 u of this round, held in the registers written above
#pragma unroll
    for (int uu = 0; uu < UH; ++uu) {
      const int u = h * UH + uu;
      const int a = q + R2 * u;
      const int al = q + R2 * uu;
      cx<T>* w = v + u * R2;
#pragma unroll
      for (int qq = 0; qq < R2; ++qq) w[qq] = slot[qq * RS + al];
      dft<R2, false, T>(w);
#pragma unroll
      for (int b = 0; b < R2; ++b) {
        if constexpr (TWS)
          w[b] = CONJ ? phase_mul_conj(w[b], kin[a + R1 * b]) : phase_mul(w[b], kin[a + R1 * b]);
        else
          w[b] = kin_mul<T, NR, CONJ>(w[b], kin[a + R1 * b]);
      }
      dft<R2, true, T>(w);
      if constexpr (TWS) w[0] = cscale(w[0], s_half);
#pragma unroll
      for (int qq = 1; qq < R2; ++qq) w[qq] = cmul_conj(w[qq], tw2[qq * (TWC > 0 ? TWC : R1) + a]);
    }
    wave_lds_sync();
#pragma unroll
    for (int uu = 0; uu < UH; ++uu) {
      const int al = q + R2 * uu;
#pragma unroll
      for (int qq = 0; qq < R2; ++qq) slot[qq * RS + al] = v[(h * UH + uu) * R2 + qq];
    }
    wave_lds_sync();
#pragma unroll
    for (int al = 0; al < RH; ++al) v[h * RH + al] = slot[q * RS + al];
  }
  dft<R1, true, T>(v);
  wave_lds_sync();
}

// -------------------------------------------------------------- C(E)
// sin(a) and 1 - cos(a).  The coupling angle per step is small in practice:
// for |a| < 1/32 the Taylor series of sin and of 1 - cos = 2 sin^2(a/2) are
// summed directly (truncation below 1e-18 relative, and no cancellation in
// 1 - cos); larger angles take an out-of-line path through the library
// sine/cosine.
// The large-angle path returns by value, so that the outputs of sin_vers
// never have their address taken (which would put them in scratch memory on
// the common path too).
struct SinVers64 { double s, v; };
struct SinVers32 { float s, v; };
__device__ __noinline__ SinVers64 sin_vers_large(double a) {
  double s, c;
  sincos(a, &s, &c);
  const double h = sin(0.5 * a);
  return {s, 2.0 * h * h};
}
__device__ __noinline__ SinVers32 sin_vers_large(float a) {
  float s, c;
  sincosf(a, &s, &c);
  const float h = sinf(0.5f * a);
  return {s, 2.0f * h * h};
}
__device__ __forceinline__ void sin_vers(double a, double* s, double* v) {
  if (fabs(a) < 0.03125) {
    const double a2 = a * a;
    // sin a = a (1 - a^2/3! + a^4/5! - a^6/7! + a^8/9!)
    double ps = 1.0 / 362880.0;
    ps = ps * a2 - 1.0 / 5040.0;
    ps = ps * a2 + 1.0 / 120.0;
    ps = ps * a2 - 1.0 / 6.0;
    *s = a + a * a2 * ps;
    // 1 - cos a = a^2/2! - a^4/4! + a^6/6! - a^8/8! + a^10/10!
    double pc = 1.0 / 3628800.0;
    pc = pc * a2 - 1.0 / 40320.0;
    pc = pc * a2 + 1.0 / 720.0;
    pc = pc * a2 - 1.0 / 24.0;
    pc = pc * a2 + 0.5;
    *v = a2 * pc;
  } else {
    const SinVers64 r = sin_vers_large(a);
    *s = r.s;
    *v = r.v;
  }
}
__device__ __forceinline__ void sin_vers(float a, float* s, float* v) {
  if (fabsf(a) < 0.125f) {
    const float a2 = a * a;
    float ps = 1.0f / 362880.0f;
    ps = ps * a2 - 1.0f / 5040.0f;
    ps = ps * a2 + 1.0f / 120.0f;
    ps = ps * a2 - 1.0f / 6.0f;
    *s = a + a * a2 * ps;
    float pc = 1.0f / 3628800.0f;
    pc = pc * a2 - 1.0f / 40320.0f;
    pc = pc * a2 + 1.0f / 720.0f;
    pc = pc * a2 - 1.0f / 24.0f;
    pc = pc * a2 + 0.5f;
    *v = a2 * pc;
  } else {
    const SinVers32 r = sin_vers_large(a);
    *s = r.s;
    *v = r.v;
  }
}


// sin and 1 - cos of the four node angles a_i = md x_i of one lane, FP32.
// The short series sin a = a - a^3/6 + a^5/120 and 1 - cos a = a^2/2 - a^4/24
// + a^6/720 are summed for every angle; their first dropped terms are below
// 1e-9 of the result for |a| < 1/8, far under FP32 rounding.  When any angle
// of the wavefront is larger (one uniform branch, not taken in practice),
// those angles are redone through the library sine and cosine.
__device__ __forceinline__ void sin_vers4(float md, const float* xk, float* sn, float* vs) {
  float a[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = md * xk[i];
    const float a2 = a[i] * a[i];
    sn[i] = __builtin_fmaf(a[i] * a2, __builtin_fmaf(a2, 1.0f / 120.0f, -1.0f / 6.0f), a[i]);
    vs[i] = a2 * __builtin_fmaf(a2, __builtin_fmaf(a2, 1.0f / 720.0f, -1.0f / 24.0f), 0.5f);
  }
  const float am = fmaxf(fmaxf(fabsf(a[0]), fabsf(a[1])), fmaxf(fabsf(a[2]), fabsf(a[3])));
  if (__builtin_expect(__ballot(!(am < 0.125f)) != 0, 0)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!(fabsf(a[i]) < 0.125f)) {
        const SinVers32 r = sin_vers_large(a[i]);
        sn[i] = r.s;
        vs[i] = r.v;
      }
    }
  }
}

// The four node angles of a contraction tile: sin_vers4 where the register
// budget allows (three waves per SIMD, n_r >= 256); at n_r <= 128 (four waves
// per SIMD, 128 registers) the four values held across its library fallback
// spill, and the angles take sin_vers one at a time.
template <int NR>
__device__ __forceinline__ void sin_vers_tile(float md, const float* xk, float* sn, float* vs) {
  if constexpr (NR >= 256) {
    sin_vers4(md, xk, sn, vs);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) sin_vers(md * xk[i], &sn[i], &vs[i]);
  }
}
template <int NR>
__device__ __forceinline__ void sin_vers_tile(double md, const double* xk, double* sn, double* vs) {
#pragma unroll
  for (int i = 0; i < 4; ++i) sin_vers(md * xk[i], &sn[i], &vs[i]);
}

// ----------------------------------------------- C(E) on the matrix cores
// Mixed form: psi += T^T (R - I) T psi over the J axis, per radial point, as
// 16x16x16 BF16 matrix-core products with FP32 accumulation.  Both operands
// are split into bf16 hi + lo parts and three products are kept
// (hi*hi + hi*lo + lo*hi).  The increment form keeps the large identity part
// of the step exact in FP32; only the small rotation increment goes through
// bf16.  One wavefront handles 16 radial points: lane l works on radial point
// r0 + l%16 and J (or node) rows 4(l/16) .. 4(l/16)+3, which is the operand
// layout of the 16x16x16 instruction, so the forward product's output is
// directly the inverse product's B operand.
// The lane index, hidden from the optimiser so that the lane-dependent
// addresses of a contraction round are recomputed there (a few integer
// operations) instead of being kept live, or spilled, across the transforms.
__device__ __forceinline__ int fresh_lane() {
  int l = static_cast<int>(threadIdx.x) & 63;
  asm volatile("" : "+v"(l));
  return l;
}

typedef short mf_short4 __attribute__((ext_vector_type(4)));
typedef float mf_float4 __attribute__((ext_vector_type(4)));

// hi = bf16(v), lo = bf16(v - hi), element by element, two elements per
// packed conversion
typedef float mf_float2 __attribute__((ext_vector_type(2)));
typedef __bf16 mf_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned int bf16x2_rne(float a, float b) {
  const mf_float2 f = {a, b};
  return __builtin_bit_cast(unsigned int, __builtin_convertvector(f, mf_bf16x2));
}
__device__ __forceinline__ void split4(const float* v, mf_short4& hi, mf_short4& lo) {
  unsigned int h[2], l[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    h[k] = bf16x2_rne(v[2 * k], v[2 * k + 1]);
    l[k] = bf16x2_rne(v[2 * k] - __uint_as_float(h[k] << 16), v[2 * k + 1] - __uint_as_float(h[k] & 0xffff0000u));
  }
  hi = __builtin_bit_cast(mf_short4, (unsigned long long)h[0] | ((unsigned long long)h[1] << 32));
  lo = __builtin_bit_cast(mf_short4, (unsigned long long)l[0] | ((unsigned long long)l[1] << 32));
}
__device__ __forceinline__ mf_float4 mma3(mf_short4 ahi, mf_short4 alo, mf_short4 bhi,
                                         mf_short4 blo, mf_float4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, c, 0, 0, 0);
  return c;
}

// Row offsets (elements from the lines' base) of a lane's four J rows
// J = j0 + step i of both states, fixed for a contraction round.  Rows
// J >= nj are the spare row after the 2 nj lines, which the kernel zeroes
// once: the operand T is zero in the columns J >= nj, so the update writes
// back the zero it loaded, and neither the loads nor the stores of a tile
// branch on J.
template <int NR, typename T>
struct CpRows {
  int g[4], e[4];
  __device__ __forceinline__ CpRows(int nj, int j0, int step) {
    const int spare = lds_row<NR, T>(2 * nj);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int J = j0 + step * i;
      g[i] = J < nj ? lds_row<NR, T>(J) : spare;
      e[i] = J < nj ? lds_row<NR, T>(nj + J) : spare;
    }
  }
};

// frag: 4 operand blocks [A_hi, A_lo, At_hi, At_lo] x 64 lanes x 4 bf16;
// x: the angle nodes padded with zeros to 16
template <int NR>
__device__ __forceinline__ void coupling_mfma(cx<float>* sh, int nj, int r0,
                                           const unsigned short* __restrict__ frag,
                                           const float* __restrict__ x,
                                           const float* __restrict__ mudt, float E) {
  using T = float;
  constexpr int NRH = NR / fwd_split<NR, float>();   // radial points of this round
  const int lane = fresh_lane();
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nwaves = (blockDim.x + 63) >> 6;
  const int col = lane & 15;
  const int rb = (lane >> 4) * 4;  // first J (inputs) / node (outputs) row of this lane
  mf_short4 Ahi, Alo, Bthi, Btlo;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Ahi[i] = static_cast<short>(frag[(0 * 64 + lane) * 4 + i]);
    Alo[i] = static_cast<short>(frag[(1 * 64 + lane) * 4 + i]);
    Bthi[i] = static_cast<short>(frag[(2 * 64 + lane) * 4 + i]);
    Btlo[i] = static_cast<short>(frag[(3 * 64 + lane) * 4 + i]);
  }
  float xk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) xk[i] = x[rb + i];   // x holds 16 nodes, zero beyond nj
  const CpRows<NR, T> rows(nj, rb, 1);
#pragma unroll 1
  for (int tile = wave; tile * 16 < NRH; tile += nwaves) {
    const int rl = tile * 16 + col;   // radial point within the round (LDS)
    const int r = r0 + rl;            // on the grid (tables)
    // psi rows J = rb..rb+3 of both states at radial point r
    float gr[4], gi[4], er[4], ei[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const cx<float> g = sh[rows.g[i] + rl], e = sh[rows.e[i] + rl];
      gr[i] = g.x; gi[i] = g.y; er[i] = e.x; ei[i] = e.y;
    }
    mf_short4 h0, l0, h1, l1, h2, l2, h3, l3;
    split4(gr, h0, l0);
    split4(gi, h1, l1);
    split4(er, h2, l2);
    split4(ei, h3, l3);
    const mf_float4 z = {0.f, 0.f, 0.f, 0.f};
    // Phi = T psi for each of (g re, g im, e re, e im); lane holds nodes rb..rb+3
    mf_float4 Pgr = mma3(Ahi, Alo, h0, l0, z);
    mf_float4 Pgi = mma3(Ahi, Alo, h1, l1, z);
    mf_float4 Per = mma3(Ahi, Alo, h2, l2, z);
    mf_float4 Pei = mma3(Ahi, Alo, h3, l3, z);
    // (R - I) Phi per node: dg = -v Phi_g + i s Phi_e, de = i s Phi_g - v Phi_e
    float sn[4], vs[4];
    sin_vers_tile<NR>(mudt[r] * E, xk, sn, vs);
    float dgr[4], dgi[4], der[4], dei[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dgr[i] = -vs[i] * Pgr[i] - sn[i] * Pei[i];
      dgi[i] = -vs[i] * Pgi[i] + sn[i] * Per[i];
      der[i] = -vs[i] * Per[i] - sn[i] * Pgi[i];
      dei[i] = -vs[i] * Pei[i] + sn[i] * Pgr[i];
    }
    split4(dgr, h0, l0);
    split4(dgi, h1, l1);
    split4(der, h2, l2);
    split4(dei, h3, l3);
    mf_float4 cgr, cgi, cer, cei;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cgr[i] = gr[i]; cgi[i] = gi[i]; cer[i] = er[i]; cei[i] = ei[i];
    }
    // psi += T^T dPhi, accumulated in FP32 on top of the exact old psi
    cgr = mma3(Bthi, Btlo, h0, l0, cgr);
    cgi = mma3(Bthi, Btlo, h1, l1, cgi);
    cer = mma3(Bthi, Btlo, h2, l2, cer);
    cei = mma3(Bthi, Btlo, h3, l3, cei);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float* og = reinterpret_cast<float*>(sh + rows.g[i] + rl);
      float* oe = reinterpret_cast<float*>(sh + rows.e[i] + rl);
      og[0] = cgr[i]; og[1] = cgi[i];
      oe[0] = cer[i]; oe[1] = cei[i];
    }
  }
}


// FP32 / FP64 forms: the same increment-form contraction on the 16x16x4
// matrix-core instructions of the working precision (no operand splitting).
// The K = 16 contraction is four instructions; instruction i sums four of
// the J (or node) rows, lane l feeding the rows it owns, and the forward
// output rows are again the inverse's operand rows.  Row ownership follows
// the instruction's output layout: lane l, element i holds row 4 (l/16) + i
// for the FP32 instruction and row 4 i + l/16 for the FP64 one.
typedef double mf_double4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaK4;
template <>
struct MfmaK4<float> {
  typedef mf_float4 acc;
  __device__ static __forceinline__ int row(int g, int i) { return 4 * g + i; }
  __device__ static __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void settle(acc&, acc&, acc&, acc&) {}
};
template <>
struct MfmaK4<double> {
  typedef mf_double4 acc;
  __device__ static __forceinline__ int row(int g, int i) { return 4 * i + g; }
  __device__ static __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // The end of a product chain: the four accumulators are taken as operands
  // of an empty statement, so that the chain is complete before any of them
  // is read and the compiler's hazard recognizer places its wait states for
  // the matrix-core result here (no explicit stall: extra waits of 16 to 96
  // states gave the same bits on the full FP64 workload).
  __device__ static __forceinline__ void settle(acc& a, acc& b, acc& c, acc& d) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
  }
};

// The J (or node) row fed by element i of lane group g: MfmaK4::row, or in
// the half-K order (N_J <= kHalfKMaxNJ, elements i < 2 only) 2g + i in FP32
// (whose fragment table is built in that order) and the same 4i + g in FP64.
template <typename T, bool KH>
__device__ __forceinline__ int mf_row(int g, int i) {
  return (KH && sizeof(T) == 4) ? 2 * g + i : MfmaK4<T>::row(g, i);
}

// frag: [2][64 lanes][4]: block 0 A_i = T[l%16][row(l/16, i)], block 1 the
// transpose T[row(l/16, i)][l%16]; zero outside nj (in the half-K order for
// FP32 when KH).  KH: N_J <= kHalfKMaxNJ, two of the four K instructions.
template <typename T, int NR, bool KH>
__device__ __forceinline__ void coupling_mfma_exact(cx<T>* sh, int nj, int r0,
                                                    const T* __restrict__ frag,
                                                    const T* __restrict__ x,
                                                    const T* __restrict__ mudt, T E) {
  typedef typename MfmaK4<T>::acc acc_t;
  constexpr int NRH = NR / fwd_split<NR, T>();
  constexpr int NK = KH ? 2 : 4;
  const int lane = fresh_lane();
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int nwaves = (blockDim.x + 63) >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  T A[4], At[4], xk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int J = mf_row<T, KH>(grp, i);
    A[i] = frag[(0 * 64 + lane) * 4 + i];
    At[i] = frag[(1 * 64 + lane) * 4 + i];
    xk[i] = (i < NK && J < nj) ? x[J] : T(0);
  }
  // this lane's rows: 4 grp + i (FP32 instruction) or 4 i + grp (FP64);
  // 2 grp + i in the FP32 half-K order
  const CpRows<NR, T> rows(nj, mf_row<T, KH>(grp, 0), mf_row<T, KH>(0, 1) - mf_row<T, KH>(0, 0));
#pragma unroll 1
  for (int tile = wave; tile * 16 < NRH; tile += nwaves) {
    const int rl = tile * 16 + col;   // radial point within the round (LDS)
    const int r = r0 + rl;            // on the grid (tables)
    const acc_t z = {T(0), T(0), T(0), T(0)};
    acc_t cgr = z, cgi = z, cer = z, cei = z;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const cx<T> g = sh[rows.g[i] + rl], e = sh[rows.e[i] + rl];
      cgr[i] = g.x; cgi[i] = g.y; cer[i] = e.x; cei[i] = e.y;
    }
    acc_t Pgr = z, Pgi = z, Per = z, Pei = z;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      Pgr = MfmaK4<T>::mma(A[i], cgr[i], Pgr);
      Pgi = MfmaK4<T>::mma(A[i], cgi[i], Pgi);
      Per = MfmaK4<T>::mma(A[i], cer[i], Per);
      Pei = MfmaK4<T>::mma(A[i], cei[i], Pei);
    }
    MfmaK4<T>::settle(Pgr, Pgi, Per, Pei);
    const T md = mudt[r] * E;
    T sn[4], vs[4];
    sin_vers_tile<NR>(md, xk, sn, vs);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const T gr = Pgr[i], gi = Pgi[i], er = Per[i], ei = Pei[i];
      Pgr[i] = -vs[i] * gr - sn[i] * ei;
      Pgi[i] = -vs[i] * gi + sn[i] * er;
      Per[i] = -vs[i] * er - sn[i] * gi;
      Pei[i] = -vs[i] * ei + sn[i] * gr;
    }
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      cgr = MfmaK4<T>::mma(At[i], Pgr[i], cgr);
      cgi = MfmaK4<T>::mma(At[i], Pgi[i], cgi);
      cer = MfmaK4<T>::mma(At[i], Per[i], cer);
      cei = MfmaK4<T>::mma(At[i], Pei[i], cei);
    }
    MfmaK4<T>::settle(cgr, cgi, cer, cei);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      T* og = reinterpret_cast<T*>(sh + rows.g[i] + rl);
      T* oe = reinterpret_cast<T*>(sh + rows.e[i] + rl);
      og[0] = cgr[i]; og[1] = cgi[i];
      oe[0] = cer[i]; oe[1] = cei[i];
    }
  }
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of four per-lane partials over the workgroup, in a fixed order.
__device__ __forceinline__ void block_sum4(double* v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wid * 4 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w * 4 + i];
      v[i] = s;
    }
  }
  __syncthreads();
}


// Absorber mask at one point: the removed probability is accumulated in
// FP64.  absorb_point_nb is the same without the branch (bit-identical: m = 1
// adds 0 and scales by 1), for the few registers that may lie in the
// absorber: one read-modify-write of the accumulator per step instead of one
// per taken branch.
template <typename T>
__device__ __forceinline__ void absorb_point_nb(cx<T>& v, T m, double& ab) {
  ab += static_cast<double>((T(1) - m * m) * norm2(v));
  v = cscale(v, m);
}
template <typename T>
__device__ __forceinline__ void absorb_point(cx<T>& v, T m, double& ab) {
  if (m != T(1)) {
    ab += static_cast<double>((T(1) - m * m) * norm2(v));
    v = cscale(v, m);
  }
}

// --------------------------------------------------------------- kernel
// Occupancy target (waves per SIMD) of the fused step.  The complex64 forms
// at n_r = 256 and 512 (three waves per molecule at J_max = 10, n_r = 256)
// run four molecules per CU within 168 VGPRs, which the LDS copy of a
// molecule also allows; at n_r <= 128 (16 values per lane) four waves per
// SIMD fit in 128 VGPRs and the LDS holds more molecules than that.  The FP64
// form is bounded by LDS (one molecule of complex128 lines per CU) and may use
// 256 VGPRs.
template <typename T, int NR>
struct MolOcc { static constexpr int waves = sizeof(T) == 8 ? 2 : (NR <= 128 ? 4 : 3); };


// coupling path: BF16 hi/lo split on 16x16x16 (mixed form) or the
// working precision on 16x16x4 (FP32 and FP64 forms)
// (kCpExactHalf: the working precision with N_J <= kHalfKMaxNJ, two of the
// four K instructions; a launch picks it from N_J, so that a kernel holds
// one contraction path)
enum { kCpExact = 0, kCpBf16x3 = 1, kCpExactHalf = 2 };

// raised wave priority over the contraction rounds (see the step loop)
template <typename T, int NR, int CP>
inline constexpr bool kPrioContraction = CP == kCpBf16x3 && NR >= 256;

// ONE: the launch advances exactly one step (the coupled step's case); the
// step loop then has no back edge, and the register allocation needs no
// spills.
template <typename T, int NR, int CP, bool ONE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MolOcc<T, NR>::waves)))
void mol_step_kernel(MolArgs a) {
  constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2;
  static_assert(CP != kCpBf16x3 || stage_tables<NR, T>(),
                "the BF16 contraction reads its operands from the LDS copy of the tables");
  extern __shared__ __align__(16) unsigned char smem[];
  const int nj = a.nj;
  const int L = 2 * nj;
  // LDS: transform tables | lines | spare row (the contractions' rows
  // J >= nj) | reduction scratch
  constexpr size_t TB = lds_table_bytes<NR, T>();
  cx<T>* kin_s = reinterpret_cast<cx<T>*>(smem);
  cx<T>* tw_s = kin_s + NR;
  T* mask_s = reinterpret_cast<T*>(tw_s + StagedTables<NR, T>::tw_elems);
  unsigned char* frag_s = smem + StagedTables<NR, T>::fft_bytes;
  float* x_s = reinterpret_cast<float*>(frag_s + StagedTables<NR, T>::frag_bytes);
  cx<T>* sh = reinterpret_cast<cx<T>*>(smem + TB);
  double* red = reinterpret_cast<double*>(smem + TB + sizeof(cx<T>) * (lds_row<NR, T>(L) + NR / fwd_split<NR, T>()));

  const int mol = blockIdx.x;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int line = tid / R2;
  const int q = tid - line * R2;
  const bool active = line < L;

  const char* ws = a.ws;
  MolTabs<T> tb;
  if constexpr (sizeof(T) == 8) {
    tb.kin = reinterpret_cast<const cx<T>*>(ws + a.lay.kin_d);
    tb.tw = reinterpret_cast<const cx<T>*>(ws + a.lay.tw_d);
    tb.vph = reinterpret_cast<const cx<T>*>(ws + a.lay.vph_d);
    tb.x = reinterpret_cast<const T*>(ws + a.lay.x_d);
    tb.mudt = reinterpret_cast<const T*>(ws + a.lay.mudt_d);
    tb.mask = reinterpret_cast<const T*>(ws + a.lay.mask_d);
  } else {
    tb.kin = reinterpret_cast<const cx<T>*>(ws + a.lay.kin_f);
    tb.tw = reinterpret_cast<const cx<T>*>(ws + (tw_scaled<NR, T>() ? a.lay.tw_fs : a.lay.tw_f));
    tb.vph = reinterpret_cast<const cx<T>*>(ws + a.lay.vph_f);
    tb.x = reinterpret_cast<const T*>(ws + a.lay.x_f);
    tb.mudt = reinterpret_cast<const T*>(ws + a.lay.mudt_f);
    tb.mask = reinterpret_cast<const T*>(ws + a.lay.mask_f);
  }
  tb.mu = reinterpret_cast<const double*>(ws + a.lay.mu_d);
  tb.cj = reinterpret_cast<const double*>(ws + a.lay.cj_d);

  // field seen by this molecule (gathered from E_x at its cell, or given);
  // a readout-only launch (no step) reads no field
  double Ed = 0.0;
  if (ONE || a.n_steps > 0) {
    if (a.Ex != nullptr) {
      const int c = a.cell_of_mol[mol];
      Ed = (a.ex_is_float ? static_cast<double>(reinterpret_cast<const float*>(a.Ex)[c])
                          : reinterpret_cast<const double*>(a.Ex)[c]) * a.inv_eau;
    } else {
      Ed = a.E_mol[mol];
    }
  }
  if (a.E_out != nullptr && tid == 0) a.E_out[mol] = Ed;
  const T E = static_cast<T>(Ed);

  // the contractions' spare row (rows J >= nj) holds zeros; the barrier
  // before the first contraction publishes them
  for (int i = tid; i < NR / fwd_split<NR, T>(); i += nthr) sh[lds_row<NR, T>(L) + i] = cx<T>{T(0), T(0)};

  cx<T>* psi = reinterpret_cast<cx<T>*>(a.psi) + static_cast<size_t>(mol) * L * NR;
  cx<T>* slot = sh + lds_row<NR, T>(line);
  const int loff = line * NR + q;  // this lane's first element of its line
  cx<T> v[R1];
  if (active) {
#pragma unroll
    for (int p = 0; p < R1; ++p) v[p] = psi[loff + R2 * p];
  }
  // the tables read at every element go to LDS (the per-element L1/L2
  // traffic and latency of these reads dominated the step otherwise)
  if constexpr (stage_tables<NR, T>()) {
    stage_tables_to_lds<NR, T>(kin_s, tw_s, mask_s, tb.kin, tb.tw, tb.mask);
    lds_stage(frag_s, ws + (CP == kCpBf16x3 ? a.lay.tmfrag : a.lay.tmfrag_f), StagedTables<NR, T>::frag_bytes);
    if (tid < StagedTables<NR, T>::x_pad) x_s[tid] = tid < nj ? static_cast<float>(tb.x[tid]) : 0.0f;
    __syncthreads();
  }

  // SP exchange rounds of NRH radial points; round h holds the registers
  // p in [h PH, (h+1) PH), i.e. r = q + R2 p in [h NRH, (h+1) NRH)
  constexpr int SP = fwd_split<NR, T>(), PH = R1 / SP, NRH = NR / SP;
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
      kin = opaque(tb.kin);
      tw = opaque(tb.tw);
      mask = opaque(tb.mask);
    }
    const cx<T>* vph = opaque(tb.vph);
    if (active) kinetic_half<T, NR, false, SP, 0, tw_scaled<NR, T>()>(v, slot, q, kin, tw);
#pragma unroll
    for (int h = 0; h < SP; ++h) {
      if (active) {
#pragma unroll
        for (int pp = 0; pp < PH; ++pp) {
          const int p = h * PH + pp;
          v[p] = phase_mul(v[p], vph[loff + R2 * p]);
          slot[q + R2 * pp] = v[p];
        }
      }
      __syncthreads();
      // in the mixed form at N_r >= 256 the contraction runs at raised wave
      // priority: a workgroup's waves wait for its slowest one at the next
      // barrier, so on a SIMD shared with other workgroups' transforms its
      // issue comes first (0.3-0.9% faster at the 100,000-molecule launch; in
      // the FP32 form it measured 0.7% slower at N_r = 256 and 1.5% at 128,
      // in FP64 the same)
      if constexpr (kPrioContraction<T, NR, CP>) __builtin_amdgcn_s_setprio(1);
      // contraction operands: from the LDS copy (complex64 forms) or the workspace
      if constexpr (CP == kCpBf16x3) {
        coupling_mfma<NR>(sh, nj, h * NRH, reinterpret_cast<const unsigned short*>(frag_s),
                          reinterpret_cast<const float*>(x_s), tb.mudt, E);
      } else if constexpr (stage_tables<NR, T>()) {
        coupling_mfma_exact<T, NR, CP == kCpExactHalf>(sh, nj, h * NRH, reinterpret_cast<const T*>(frag_s),
                                                       reinterpret_cast<const T*>(x_s), tb.mudt, E);
      } else {
        const T* frag = reinterpret_cast<const T*>(ws + (sizeof(T) == 8 ? a.lay.tmfrag_d : a.lay.tmfrag_f));
        coupling_mfma_exact<T, NR, CP == kCpExactHalf>(sh, nj, h * NRH, frag, tb.x, tb.mudt, E);
      }
      if constexpr (kPrioContraction<T, NR, CP>) __builtin_amdgcn_s_setprio(0);
      __syncthreads();
      if (active) {
#pragma unroll
        for (int pp = 0; pp < PH; ++pp) {
          const int p = h * PH + pp;
          v[p] = phase_mul(slot[q + R2 * pp], vph[loff + R2 * p]);
        }
      }
    }
    if (active) {
      kinetic_half<T, NR, false, SP, 0, tw_scaled<NR, T>()>(v, slot, q, kin, tw);
      // absorber: when it lies within the last quarter of the grid only
      // those registers are tested (one uniform branch), otherwise all
      constexpr int P0 = (3 * R1) / 4;
      if (a.kmask >= R2 * P0) {
#pragma unroll
        for (int p = P0; p < R1; ++p) absorb_point_nb(v[p], mask[q + R2 * p], ab);
      } else {
#pragma unroll
        for (int p = 0; p < R1; ++p) absorb_point(v[p], mask[q + R2 * p], ab);
      }
    }
  }

  // readouts of the final state (the norm also when no dipole is asked
  // for, as the finiteness check)
  double nrm = 0.0, yld = 0.0, dd = 0.0;
  const bool want_n = a.want_norm || !a.want_d;
  if (active && (want_n || a.want_yield)) {
#pragma unroll
    for (int p = 0; p < R1; ++p) {
      const int r = q + R2 * p;
      const double n2 = static_cast<double>(norm2(v[p]));
      nrm += n2;
      if (r >= a.kdiss) yld += n2;
    }
  }
  if (a.want_d) {
    // d = 2 dr sum_r mu(r) sum_J c_J Re[conj(g_J) e_{J+1} + conj(g_{J+1}) e_J],
    // one round of radial points at a time; the J sum in the working
    // precision, the r sum in FP64
#pragma unroll
    for (int h = 0; h < SP; ++h) {
      if (h > 0) __syncthreads();   // the previous round's readers are done
      if (active) {
#pragma unroll
        for (int pp = 0; pp < PH; ++pp) slot[q + R2 * pp] = v[h * PH + pp];
      }
      __syncthreads();
      for (int rl = tid; rl < NRH; rl += nthr) {
        T acc = T(0);
        cx<T> g0 = sh[rl], e0 = sh[lds_row<NR, T>(nj) + rl];
        for (int J = 0; J + 1 < nj; ++J) {
          const cx<T> g1 = sh[lds_row<NR, T>(J + 1) + rl], e1 = sh[lds_row<NR, T>(nj + J + 1) + rl];
          const T t = g0.x * e1.x + g0.y * e1.y + g1.x * e0.x + g1.y * e0.y;
          acc += static_cast<T>(tb.cj[J]) * t;
          g0 = g1;
          e0 = e1;
        }
        dd += tb.mu[h * NRH + rl] * static_cast<double>(acc);
      }
    }
  }
  double sums[4] = {ab, nrm, yld, dd};
  block_sum4(sums, red);
  if (tid == 0) {
    const double dr = a.dr;
    const double absorbed = a.absorbed[mol] + sums[0] * dr;
    if (n_steps > 0) a.absorbed[mol] = absorbed;
    const double d = 2.0 * dr * sums[3];
    if (a.want_d && a.d_mol) a.d_mol[mol] = d;
    if (a.want_norm && a.norm_mol) a.norm_mol[mol] = sums[1] * dr;
    if (a.want_yield && a.yield_mol) a.yield_mol[mol] = sums[2] * dr + absorbed;
    if (!isfinite(d) || !isfinite(sums[1]) || !isfinite(absorbed)) atomicOr(a.status, 1);
  }
  if (active && n_steps > 0) {
    cx<T>* out = a.psi_out ? reinterpret_cast<cx<T>*>(a.psi_out) + static_cast<size_t>(mol) * L * NR : psi;
#pragma unroll
    for (int p = 0; p < R1; ++p) out[loff + R2 * p] = v[p];
  }
}

template <typename T, int NR, int CP, bool ONE>
int launch_mol_t1(const MolArgs& a, hipStream_t s) {
  static_assert(NR == FftShape<NR, T>::R1 * FftShape<NR, T>::R2, "FFT shape");
  constexpr int R2 = FftShape<NR, T>::R2;
  const int L = 2 * a.nj;
  int threads = ((L * R2 + 63) / 64) * 64;
  if (threads < 64) threads = 64;
  const size_t shm = lds_table_bytes<NR, T>() +
                     sizeof(cx<T>) * (static_cast<size_t>(lds_line_start(L, fwd_line_stride<NR, T>(), sizeof(cx<T>))) +
                                      NR / fwd_split<NR, T>()) +
                     16 * 4 * sizeof(double);
  static std::atomic<unsigned long long> lds_set{0};
  if (shm > 64 * 1024) {
    const hipError_t e = allow_large_lds(reinterpret_cast<const void*>(&mol_step_kernel<T, NR, CP, ONE>), lds_set);
    if (e != hipSuccess) return static_cast<int>(e);
  }
  hipLaunchKernelGGL((mol_step_kernel<T, NR, CP, ONE>), dim3(a.n_mol), dim3(threads), shm, s, a);
  return static_cast<int>(hipGetLastError());
}

// complex64 forms: a single-step instantiation (no spills at N_r = 256,
// 4% faster); the FP64 form measured no gain from it
template <typename T, int NR, int CP>
int launch_mol_t(const MolArgs& a, hipStream_t s) {
  if constexpr (CP == kCpExact) {
    if (a.nj <= kHalfKMaxNJ) return launch_mol_t<T, NR, kCpExactHalf>(a, s);
  }
  if constexpr (sizeof(T) == 4) {
    if (a.n_steps == 1) return launch_mol_t1<T, NR, CP, true>(a, s);
  }
  return launch_mol_t1<T, NR, CP, false>(a, s);
}

template <typename T, int CP>
int launch_mol_any(const MolArgs& a, int n_r, hipStream_t s) {
  switch (n_r) {
    case 64: return launch_mol_t<T, 64, CP>(a, s);
    case 128: return launch_mol_t<T, 128, CP>(a, s);
    case 256: return launch_mol_t<T, 256, CP>(a, s);
    case 512: return launch_mol_t<T, 512, CP>(a, s);
    default: return static_cast<int>(hipErrorInvalidValue);
  }
}

}  // namespace msqd
