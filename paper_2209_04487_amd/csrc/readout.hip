// Readouts beside the molecular step.
//  - Excited-state radial moments of every wavepacket (Eq. (8)): per molecule
//    <chi_e|R|chi_e> = sum_{J,k} r_k |psi_e,J(r_k)|^2 dr and <chi_e|chi_e>,
//    accumulated in FP64, plus the ensemble sums over molecules and their
//    ratio in a fixed order.  One workgroup per molecule; the excited-state
//    lines are one contiguous [nj][n_r] block of the molecule-major layout.
//  - Ensemble sums of per-molecule FP64 values (dipole, norm, yield) in a
//    fixed two-stage order.
//  - Transmission, reflection and absorption spectra from monitor fluxes.
#include <hip/hip_runtime.h>

#include "readout.h"

namespace msqd {

constexpr int kRdThreads = 256;

template <typename T>
__global__ __launch_bounds__(kRdThreads) void excited_r_kernel(RdArgs a) {
  __shared__ double s_num[kRdThreads];
  __shared__ double s_pop[kRdThreads];
  const int mol = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t line = static_cast<size_t>(a.nj) * a.n_r;
  const T* pe = static_cast<const T*>(a.psi) + 2 * (static_cast<size_t>(mol) * 2 * line + line);
  double num = 0.0, pop = 0.0;
  for (size_t i = tid; i < line; i += kRdThreads) {
    const int k = static_cast<int>(i % a.n_r);
    const double re = static_cast<double>(pe[2 * i]), im = static_cast<double>(pe[2 * i + 1]);
    const double p2 = re * re + im * im;
    pop += p2;
    num += (a.r_min + k * a.dr) * p2;
  }
  s_num[tid] = num;
  s_pop[tid] = pop;
  __syncthreads();
  for (int w = kRdThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_num[tid] += s_num[tid + w];
      s_pop[tid] += s_pop[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.r_num[mol] = s_num[0] * a.dr;
    a.pop[mol] = s_pop[0] * a.dr;
  }
}

// ensemble sums over molecules (one workgroup, fixed order) and their ratio
__global__ __launch_bounds__(kRdThreads) void pair_sum_kernel(const double* x, const double* y, int n,
                                                            double* out) {
  __shared__ double sx[kRdThreads];
  __shared__ double sy[kRdThreads];
  const int tid = threadIdx.x;
  double ax = 0.0, ay = 0.0;
  for (int i = tid; i < n; i += kRdThreads) {
    ax += x[i];
    ay += y[i];
  }
  sx[tid] = ax;
  sy[tid] = ay;
  __syncthreads();
  for (int w = kRdThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      sx[tid] += sx[tid + w];
      sy[tid] += sy[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = sx[0];
    out[1] = sy[0];
    out[2] = sx[0] / sy[0];   // NaN while the excited population is exactly zero
  }
}

// stage one: block b sums molecules [b kSumBlock, (b+1) kSumBlock), thread t
// taking b kSumBlock + t + kRdThreads q, q = 0..3, then a fixed tree
__global__ __launch_bounds__(kRdThreads) void block_sums_kernel(SumArgs a) {
  __shared__ double sh[kMaxSumVecs][kRdThreads];
  const int tid = threadIdx.x;
  const int base = blockIdx.x * kSumBlock;
  for (int v = 0; v < a.nv; ++v) {
    double acc = 0.0;
    for (int q = 0; q < kSumBlock / kRdThreads; ++q) {
      const int i = base + tid + q * kRdThreads;
      if (i < a.n) acc += a.src[v][static_cast<size_t>(i) * a.stride[v]];
    }
    sh[v][tid] = acc;
  }
  __syncthreads();
  for (int w = kRdThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int v = 0; v < a.nv; ++v) sh[v][tid] += sh[v][tid + w];
    __syncthreads();
  }
  if (tid < a.nv) a.partial[static_cast<size_t>(blockIdx.x) * a.nv + tid] = sh[tid][0];
}

// stage two: one workgroup over the partials, thread t taking blocks
// t, t + kRdThreads, ..., then the same tree
__global__ __launch_bounds__(kRdThreads) void partial_sums_kernel(SumArgs a, int nblk) {
  __shared__ double sh[kMaxSumVecs][kRdThreads];
  const int tid = threadIdx.x;
  for (int v = 0; v < a.nv; ++v) {
    double acc = 0.0;
    for (int b = tid; b < nblk; b += kRdThreads) acc += a.partial[static_cast<size_t>(b) * a.nv + v];
    sh[v][tid] = acc;
  }
  __syncthreads();
  for (int w = kRdThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int v = 0; v < a.nv; ++v) sh[v][tid] += sh[v][tid + w];
    __syncthreads();
  }
  if (tid < a.nv) a.out[tid] = sh[tid][0];
}

__global__ void spectra_kernel(const double* st, const double* si, const double* sr, int n, double* tra) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const double ref = sr[f];
  tra[f] = st[f] / ref;
  tra[n + f] = (ref - si[f]) / ref;
  tra[2 * n + f] = (si[f] - st[f]) / ref;
}

int launch_excited_r(const RdArgs& a, bool f32, hipStream_t s) {
  if (a.n_mol <= 0) return 0;
  if (f32)
    hipLaunchKernelGGL(excited_r_kernel<float>, dim3(a.n_mol), dim3(kRdThreads), 0, s, a);
  else
    hipLaunchKernelGGL(excited_r_kernel<double>, dim3(a.n_mol), dim3(kRdThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.sums == nullptr) return static_cast<int>(e);
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(kRdThreads), 0, s, a.r_num, a.pop, a.n_mol, a.sums);
  return static_cast<int>(hipGetLastError());
}

int launch_ensemble_sums(const SumArgs& a, hipStream_t s) {
  const int nblk = sum_blocks(a.n);
  if (nblk > 0) {
    hipLaunchKernelGGL(block_sums_kernel, dim3(nblk), dim3(kRdThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return static_cast<int>(e);
  }
  hipLaunchKernelGGL(partial_sums_kernel, dim3(1), dim3(kRdThreads), 0, s, a, nblk);
  return static_cast<int>(hipGetLastError());
}

int launch_spectra(const double* s_trans, const double* s_inc, const double* s_ref, int n_freq, double* tra,
                   hipStream_t s) {
  if (n_freq <= 0) return 0;
  hipLaunchKernelGGL(spectra_kernel, dim3((n_freq + 255) / 256), dim3(256), 0, s, s_trans, s_inc, s_ref, n_freq,
                     tra);
  return static_cast<int>(hipGetLastError());
}

}  // namespace msqd
