// Excited-state radial moments of every wavepacket (Eq. (8)): per molecule
// <chi_e|R|chi_e> = sum_{J,k} r_k |psi_e,J(r_k)|^2 dr and <chi_e|chi_e>,
// accumulated in FP64, plus the ensemble sums over molecules in a fixed
// order.  One workgroup per molecule; the excited-state lines are one
// contiguous [nj][n_r] block of the molecule-major layout.
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

// ensemble sums over molecules (one workgroup, fixed order)
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
  }
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

}  // namespace msqd
