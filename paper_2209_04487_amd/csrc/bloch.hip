// Frozen two-level emitters (the paper's Bloch-equation comparison in the
// section on molecular mapping), one thread per emitter, classical RK4 with
// the field held over the step.  In atomic units, V = -mu E:
//   d rho_ee/dt = 2 V Im(rho_ge) - g1 rho_ee
//   d rho_ge/dt = (i w0 - g2) rho_ge - i V (2 rho_ee - 1)
// State planes [3][n] (structure of arrays: each plane is read with unit
// stride across the wavefront).
#include <hip/hip_runtime.h>

#include "bloch.h"

namespace msqd {

template <typename T>
struct BlochRhs {
  T w0, g1, g2, V;
  __device__ __forceinline__ void operator()(T pe, T u, T v, T& dpe, T& du, T& dv) const {
    dpe = T(2) * V * v - g1 * pe;
    du = -w0 * v - g2 * u;
    dv = w0 * u - g2 * v - V * (T(2) * pe - T(1));
  }
};

template <typename T>
__global__ __launch_bounds__(256) void bloch_kernel(BlochArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double Ed;
  if (a.Ex != nullptr) {
    const int c = a.cell_of_mol[i];
    Ed = (a.ex_is_float ? static_cast<double>(static_cast<const float*>(a.Ex)[c])
                        : static_cast<const double*>(a.Ex)[c]) * a.inv_eau;
  } else {
    Ed = a.E[i];
  }
  if (a.E_out) a.E_out[i] = Ed;
  T* st = static_cast<T*>(a.state);
  const size_t n = static_cast<size_t>(a.n);
  T pe = st[i], u = st[n + i], v = st[2 * n + i];
  BlochRhs<T> f{static_cast<T>(a.w0), static_cast<T>(a.g1), static_cast<T>(a.g2),
                static_cast<T>(-a.mu * Ed)};
  const T h = static_cast<T>(a.dt), h2 = h * T(0.5), h6 = h / T(6);
  for (int s = 0; s < a.n_steps; ++s) {
    T k1p, k1u, k1v, k2p, k2u, k2v, k3p, k3u, k3v, k4p, k4u, k4v;
    f(pe, u, v, k1p, k1u, k1v);
    f(pe + h2 * k1p, u + h2 * k1u, v + h2 * k1v, k2p, k2u, k2v);
    f(pe + h2 * k2p, u + h2 * k2u, v + h2 * k2v, k3p, k3u, k3v);
    f(pe + h * k3p, u + h * k3u, v + h * k3v, k4p, k4u, k4v);
    pe += h6 * (k1p + T(2) * k2p + T(2) * k3p + k4p);
    u += h6 * (k1u + T(2) * k2u + T(2) * k3u + k4u);
    v += h6 * (k1v + T(2) * k2v + T(2) * k3v + k4v);
  }
  if (a.n_steps > 0) {
    st[i] = pe;
    st[n + i] = u;
    st[2 * n + i] = v;
  }
  if (a.d) a.d[i] = 2.0 * a.mu * static_cast<double>(u);
}

int launch_bloch(const BlochArgs& a, bool f32, hipStream_t s) {
  if (a.n <= 0) return 0;
  const int blocks = (a.n + 255) / 256;
  if (f32)
    hipLaunchKernelGGL(bloch_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(bloch_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
  return static_cast<int>(hipGetLastError());
}

}  // namespace msqd
