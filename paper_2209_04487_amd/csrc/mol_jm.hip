// The molecular step in the full rotational basis j <= 1 (all m) with all
// three field components (Eq. (3) with the X, Y, Z direction cosines of the
// molecular axis).  Per electronic state four lines b = j^2 + m + j:
// (0,0), (1,-1), (1,0), (1,1); one workgroup per molecule.
//
// The coupling exp(i mu12(r) dt sigma_x (x) A), A = sum_c E_c D_c, has a
// closed form on this basis.  A only connects (0,0) with the j = 1 states:
// A|00> = |v> = sum_b v_b |b>, A|b> = conj(v_b)|00>, with
// v = ((E_x + i E_y)/sqrt6, E_z/sqrt3, (-E_x + i E_y)/sqrt6), so that
// A^2 = a^2 P, a^2 = |E|^2/3, P the projector on span{|00>, |v>}, and
//   exp(i phi sigma_x (x) A) = 1 - (1 - cos(phi a)) P + i (sin(phi a)/a) sigma_x (x) A.
// The dipole is d_c = 2 dr sum_r mu12 Re <g(r)| D_c |e(r)> with
// D_c|00> = sum_b w_cb |b>: w_x = (1, 0, -1)/sqrt6, w_y = (i, 0, i)/sqrt6,
// w_z = (0, 1, 0)/sqrt3.
#include <hip/hip_runtime.h>

#include "mol_impl.h"

namespace msqd {

namespace {

constexpr double kInvSqrt6 = 0.40824829046386301637;
constexpr double kInvSqrt3 = 0.57735026918962576451;

template <typename T>
__device__ __forceinline__ cx<T> cconj_mul(cx<T> a, cx<T> b) {  // conj(a) * b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.y, a.x}; }

// The three factors of the closed form at one radial point, x = phi a:
// vs = 1 - cos x, f = sin(x) / a, wv = (1 - cos x) / a^2.  For small |x| they
// come from the series of sin(x)/x and (1 - cos x)/x^2 times phi and phi^2,
// which needs no division and stays finite as the field goes to zero; larger
// angles use the library sine and the per-molecule reciprocals of a and a^2
// (a is then far from zero).
__device__ __forceinline__ void sinc_versc(double x2, double* sc, double* vc) {
  double ps = 1.0 / 362880.0;
  ps = ps * x2 - 1.0 / 5040.0;
  ps = ps * x2 + 1.0 / 120.0;
  ps = ps * x2 - 1.0 / 6.0;
  *sc = 1.0 + x2 * ps;
  double pc = 1.0 / 3628800.0;
  pc = pc * x2 - 1.0 / 40320.0;
  pc = pc * x2 + 1.0 / 720.0;
  pc = pc * x2 - 1.0 / 24.0;
  *vc = pc * x2 + 0.5;
}
__device__ __forceinline__ void sinc_versc(float x2, float* sc, float* vc) {
  float ps = 1.0f / 362880.0f;
  ps = ps * x2 - 1.0f / 5040.0f;
  ps = ps * x2 + 1.0f / 120.0f;
  ps = ps * x2 - 1.0f / 6.0f;
  *sc = 1.0f + x2 * ps;
  float pc = 1.0f / 3628800.0f;
  pc = pc * x2 - 1.0f / 40320.0f;
  pc = pc * x2 + 1.0f / 720.0f;
  pc = pc * x2 - 1.0f / 24.0f;
  *vc = pc * x2 + 0.5f;
}
template <typename T>
__device__ __forceinline__ void jm_factors(T phi, T a, T inv_a, T inv_a2, T* vs, T* f, T* wv) {
  const T x = phi * a;
  const T lim = sizeof(T) == 8 ? T(0.03125) : T(0.125);
  if (fabs(x) < lim) {
    T sc, vc;
    sinc_versc(x * x, &sc, &vc);
    *f = phi * sc;
    *wv = (phi * phi) * vc;
    *vs = (x * x) * vc;
  } else {
    T sn, v;
    sin_vers(x, &sn, &v);
    *f = sn * inv_a;
    *wv = v * inv_a2;
    *vs = v;
  }
}

// exp(i phi sigma_x (x) A) at one radial point: g, e hold the four (j, m)
// amplitudes of each state
template <typename T>
__device__ __forceinline__ void coupling_jm_point(cx<T>* g, cx<T>* e, const cx<T>* v, T a, T inv_a, T inv_a2,
                                                  T phi) {
  T vs, f, wv;
  jm_factors(phi, a, inv_a, inv_a2, &vs, &f, &wv);
  cx<T> vg = {T(0), T(0)}, ve = {T(0), T(0)};  // <v|g_1>, <v|e_1>
#pragma unroll
  for (int b = 1; b < 4; ++b) {
    vg = vg + cconj_mul(v[b - 1], g[b]);
    ve = ve + cconj_mul(v[b - 1], e[b]);
  }
  const cx<T> g0 = g[0], e0 = e[0];
  g[0] = g0 - cscale(g0, vs) + cscale(times_i(ve), f);
  e[0] = e0 - cscale(e0, vs) + cscale(times_i(vg), f);
#pragma unroll
  for (int b = 1; b < 4; ++b) {
    const cx<T> vb = v[b - 1];
    g[b] = g[b] - cscale(cmul(vb, vg), wv) + cscale(times_i(cmul(vb, e0)), f);
    e[b] = e[b] - cscale(cmul(vb, ve), wv) + cscale(times_i(cmul(vb, g0)), f);
  }
}

}  // namespace

// Same work decomposition as the m = 0 step (mol_impl.h): lanes own radial
// columns of one line for the transforms, and complex64 lines go through LDS
// in two rounds of half the radial points, the pointwise coupling included.
// The tables are staged in the compact layout (complex64 forms), which keeps
// a workgroup small enough for ten molecules per CU.
// Occupancy target: three waves per SIMD for the complex64 form (168
// registers); the complex128 form takes what it needs.
template <typename T>
struct JmOcc { static constexpr int waves = sizeof(T) == 4 ? 3 : 1; };

// ONE: the launch advances exactly one step (as in the m = 0 kernel).
template <typename T, int NR, bool ONE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(JmOcc<T>::waves))) void mol_jm_kernel(MolArgs a) {
  constexpr int R1 = FftShape<NR, T>::R1, R2 = FftShape<NR, T>::R2;
  constexpr int NB = 4, L = 2 * NB;
  constexpr int SP = fwd_split<NR, T>(), PH = R1 / SP, NRH = NR / SP;
  typedef StagedTables<NR, T, true, false> TBL;
  constexpr size_t TB = TBL::bytes;
  extern __shared__ __align__(16) unsigned char smem[];
  cx<T>* kin_s = reinterpret_cast<cx<T>*>(smem);
  cx<T>* tw_s = kin_s + NR;
  T* mask_s = reinterpret_cast<T*>(tw_s + TBL::tw_elems);
  cx<T>* sh = reinterpret_cast<cx<T>*>(smem + TB);
  double* red = reinterpret_cast<double*>(smem + TB + sizeof(cx<T>) * lds_row<NR, T>(L));

  const int mol = blockIdx.x;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int line = tid / R2;            // blockDim = L * R2: every thread holds a line
  const int q = tid - line * R2;
  const int st = line / NB, b = line - st * NB, jl = b == 0 ? 0 : 1;

  const char* ws = a.ws;
  const bool dbl = sizeof(T) == 8;
  const cx<T>* kin_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.kin_d : a.lay.kin_f));
  const cx<T>* tw_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.tw_d : a.lay.tw_f));
  const cx<T>* vph_g = reinterpret_cast<const cx<T>*>(ws + (dbl ? a.lay.vph_d : a.lay.vph_f));
  const T* mudt = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mudt_d : a.lay.mudt_f));
  const T* mask_g = reinterpret_cast<const T*>(ws + (dbl ? a.lay.mask_d : a.lay.mask_f));
  const double* mu = reinterpret_cast<const double*>(ws + a.lay.mu_d);

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
  const cx<T> v[3] = {{static_cast<T>(E3[0] * kInvSqrt6), static_cast<T>(E3[1] * kInvSqrt6)},
                      {static_cast<T>(E3[2] * kInvSqrt3), T(0)},
                      {static_cast<T>(-E3[0] * kInvSqrt6), static_cast<T>(E3[1] * kInvSqrt6)}};
  const double a2d = (E3[0] * E3[0] + E3[1] * E3[1] + E3[2] * E3[2]) / 3.0;
  const T aa = static_cast<T>(sqrt(a2d));
  // reciprocals for the large-angle branch only (|phi a| >= 1/32 there)
  const T inv_a = a2d > 0.0 ? static_cast<T>(1.0 / sqrt(a2d)) : T(0);
  const T inv_a2 = a2d > 0.0 ? static_cast<T>(1.0 / a2d) : T(0);

  cx<T>* psi = reinterpret_cast<cx<T>*>(a.psi) + static_cast<size_t>(mol) * L * NR;
  cx<T>* slot = sh + lds_row<NR, T>(line);
  const int loff = line * NR + q;
  const int voff = (st * a.nj + jl) * NR + q;   // potential phases depend on (state, j)
  cx<T> vv[R1];
#pragma unroll
  for (int p = 0; p < R1; ++p) vv[p] = psi[loff + R2 * p];
  if constexpr (stage_tables<NR, T>()) {
    stage_tables_to_lds<NR, T, true>(kin_s, tw_s, mask_s, kin_g, tw_g, mask_g);
    __syncthreads();
  }

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
        slot[q + R2 * pp] = phase_mul(vv[p], vph[voff + R2 * p]);
      }
      __syncthreads();
      for (int rl = tid; rl < NRH; rl += nthr) {
        cx<T> g[NB], e[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          g[k] = sh[lds_row<NR, T>(k) + rl];
          e[k] = sh[lds_row<NR, T>(NB + k) + rl];
        }
        coupling_jm_point(g, e, v, aa, inv_a, inv_a2, mudt[h * NRH + rl]);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          sh[lds_row<NR, T>(k) + rl] = g[k];
          sh[lds_row<NR, T>(NB + k) + rl] = e[k];
        }
      }
      __syncthreads();
#pragma unroll
      for (int pp = 0; pp < PH; ++pp) {
        const int p = h * PH + pp;
        vv[p] = phase_mul(slot[q + R2 * pp], vph[voff + R2 * p]);
      }
    }
    kinetic_half<T, NR, false, SP, TBL::TWC>(vv, slot, q, kin, tw);
    // absorber: when it lies within the last quarter of the grid only those
    // registers are tested (one uniform branch), otherwise all
    constexpr int P0 = (3 * R1) / 4;
    if (a.kmask >= R2 * P0) {
#pragma unroll
      for (int p = P0; p < R1; ++p) absorb_point_nb(vv[p], mask[q + R2 * p], ab);
    } else {
#pragma unroll
      for (int p = 0; p < R1; ++p) absorb_point(vv[p], mask[q + R2 * p], ab);
    }
  }

  // readouts: norm, yield, and the dipole vector (in the same rounds of
  // radial points)
  double nrm = 0.0, yld = 0.0;
#pragma unroll
  for (int p = 0; p < R1; ++p) {
    const double n2 = static_cast<double>(norm2(vv[p]));
    nrm += n2;
    if (q + R2 * p >= a.kdiss) yld += n2;
  }
  double dc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int h = 0; h < SP; ++h) {
    __syncthreads();   // the previous users of the slots are done
#pragma unroll
    for (int pp = 0; pp < PH; ++pp) slot[q + R2 * pp] = vv[h * PH + pp];
    __syncthreads();
    for (int rl = tid; rl < NRH; rl += nthr) {
      cx<double> g[NB], e[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const cx<T> gt = sh[lds_row<NR, T>(k) + rl], et = sh[lds_row<NR, T>(NB + k) + rl];
        g[k] = {static_cast<double>(gt.x), static_cast<double>(gt.y)};
        e[k] = {static_cast<double>(et.x), static_cast<double>(et.y)};
      }
      // Re[conj(g0) <w|e_1> + <g_1|w> e0] for w_x, w_y, w_z
      const cx<double> ex_ = {(e[1].x - e[3].x) * kInvSqrt6, (e[1].y - e[3].y) * kInvSqrt6};   // <w_x|e_1>
      const cx<double> gx_ = {(g[1].x - g[3].x) * kInvSqrt6, -(g[1].y - g[3].y) * kInvSqrt6};  // <g_1|w_x>
      // <w_y|e_1> = -i (e_-1 + e_+1)/sqrt6 ; <g_1|w_y> = i conj(g_-1 + g_+1)/sqrt6
      const cx<double> ey_ = {(e[1].y + e[3].y) * kInvSqrt6, -(e[1].x + e[3].x) * kInvSqrt6};
      const cx<double> gy_ = {(g[1].y + g[3].y) * kInvSqrt6, (g[1].x + g[3].x) * kInvSqrt6};
      const double tx = (g[0].x * ex_.x + g[0].y * ex_.y) + (gx_.x * e[0].x - gx_.y * e[0].y);
      const double ty = (g[0].x * ey_.x + g[0].y * ey_.y) + (gy_.x * e[0].x - gy_.y * e[0].y);
      const double tz = kInvSqrt3 * ((g[0].x * e[2].x + g[0].y * e[2].y) + (g[2].x * e[0].x + g[2].y * e[0].y));
      const double m = mu[h * NRH + rl];
      dc[0] += m * tx;
      dc[1] += m * ty;
      dc[2] += m * tz;
    }
  }
  // workgroup sums of (ab, nrm, yld, dx, dy, dz) in a fixed order
  double vals[6] = {ab, nrm, yld, dc[0], dc[1], dc[2]};
  const int lane = tid & 63, wid = tid >> 6, nw = (nthr + 63) >> 6;
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

// LDS bytes of one (j, m) workgroup: staged tables, the eight line slots,
// and the reduction scratch
template <typename T, int NR>
constexpr size_t jm_lds_bytes() {
  return StagedTables<NR, T, true, false>::bytes +
         sizeof(cx<T>) * static_cast<size_t>(lds_line_start(8, fwd_line_stride<NR, T>(), sizeof(cx<T>))) +
         6 * 16 * sizeof(double);
}

template <typename T, int NR, bool ONE>
int launch_jm_t1(const MolArgs& a, hipStream_t s) {
  constexpr int R2 = FftShape<NR, T>::R2;
  const int threads = 8 * R2;
  const size_t shm = jm_lds_bytes<T, NR>();
  if (shm > mol_lds_limit()) return static_cast<int>(hipErrorInvalidValue);
  static std::atomic<unsigned long long> lds_set{0};
  if (shm > 64 * 1024) {
    const hipError_t e = allow_large_lds(reinterpret_cast<const void*>(&mol_jm_kernel<T, NR, ONE>), lds_set);
    if (e != hipSuccess) return static_cast<int>(e);
  }
  hipLaunchKernelGGL((mol_jm_kernel<T, NR, ONE>), dim3(a.n_mol), dim3(threads), shm, s, a);
  return static_cast<int>(hipGetLastError());
}

// complex64: a single-step instantiation for the coupled step's launches
template <typename T, int NR>
int launch_jm_t(const MolArgs& a, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (a.n_steps == 1) return launch_jm_t1<T, NR, true>(a, s);
  }
  return launch_jm_t1<T, NR, false>(a, s);
}

template <typename T>
int launch_jm_any(const MolArgs& a, int n_r, hipStream_t s) {
  switch (n_r) {
    case 64: return launch_jm_t<T, 64>(a, s);
    case 128: return launch_jm_t<T, 128>(a, s);
    case 256: return launch_jm_t<T, 256>(a, s);
    case 512: return launch_jm_t<T, 512>(a, s);
    default: return static_cast<int>(hipErrorInvalidValue);
  }
}

int launch_mol_jm(const MolArgs& a, int n_r, bool f32, hipStream_t s) {
  return f32 ? launch_jm_any<float>(a, n_r, s) : launch_jm_any<double>(a, n_r, s);
}

}  // namespace msqd
