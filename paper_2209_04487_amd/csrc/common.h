// Internal helpers shared by the HIP sources of libmsqd: complex arithmetic,
// compile-time twiddles, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/msqd.h"

namespace msqd {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

#define MSQD_HIP(call)                                   \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return check_hip(_e, #call);   \
  } while (0)

// -------------------------------------------------------------- constants
// CODATA 2018
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kEta0 = 376.730313668;
constexpr double kEau = 5.14220674763e11;      // V/m per atomic unit of field
constexpr double kEa0 = 8.4783536255e-30;      // C m per e a0
constexpr double kTau = 2.4188843265857e-17;    // s per atomic unit of time
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------ complex type
template <typename T>
struct cx {
  T x, y;  // real, imaginary
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by +i / -i
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }

// Start (in elements) of line `line` of a molecule's LDS line array, line
// stride ls elements of el_bytes each.  complex64 rows are staggered by 16
// elements on every other group of four lines (plus 32 every eight lines) so
// that the four J rows one matrix-core operand load reads (J = 4g + i,
// g = 0..3) fall on both halves of the 64 LDS banks instead of one; the
// in-line transposes keep their two-pass access.
constexpr int lds_line_start(int line, int ls, int el_bytes) {
  return el_bytes == 8 ? line * ls + 16 * ((line >> 2) & 1) + 32 * (line >> 3) : line * ls;
}

// Rotation v * exp(i phi) as three shears (lifting): x += p y; y += u x;
// x += p y, with p = -tan(phi / 2) and u = sin(phi).  The shears have
// determinant one whatever p and u are rounded to, so the rounded product
// changes |v|^2 only at second order in the rounding of the parameters when
// averaged over the phase of v.  A rounded (cos, sin) pair instead scales
// every |v|^2 by the same factor |c + i s|^2 = 1 + O(eps), which, applied to
// every element in every step, turns into a systematic drift of the norm.
template <typename T>
__host__ __device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> lift_rot(cx<T> v, T p, T u) {
  const T x1 = fma_t(p, v.y, v.x);
  const T y1 = fma_t(u, x1, v.y);
  return {fma_t(p, y1, x1), y1};
}

// ------------------------------------------------ compile-time cos / sin
// cos(2 pi j / n) and sin(2 pi j / n) evaluated in constant expressions:
// reduce to the first octant by symmetry, then Taylor series to convergence.
constexpr double ct_taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// angle 2 pi j / n with 0 <= j < n, via octants of 8j/n
constexpr void ct_sincos_frac(long j, long n, double* s, double* c) {
  j %= n;
  if (j < 0) j += n;
  // quadrant q and remainder: angle = q*pi/2 + (j - q n/4) 2pi/n, done in rationals
  long num = 4 * j;            // angle / (pi/2) = 4j/n
  long q = num / n;            // quadrant 0..3
  long rem = num - q * n;      // remainder in [0, n): angle' = rem/n * pi/2
  double sa = 0.0, ca = 0.0;
  if (2 * rem <= n) {
    double a = (static_cast<double>(rem) / static_cast<double>(n)) * (kPi / 2.0);
    sa = ct_taylor_sin(a);
    ca = ct_taylor_cos(a);
  } else {
    double a = (static_cast<double>(n - rem) / static_cast<double>(n)) * (kPi / 2.0);
    sa = ct_taylor_cos(a);
    ca = ct_taylor_sin(a);
  }
  switch (q) {
    case 0: *s = sa; *c = ca; break;
    case 1: *s = ca; *c = -sa; break;
    case 2: *s = -sa; *c = -ca; break;
    default: *s = -ca; *c = sa; break;
  }
}

// exp(+-2 pi i j / N) split into k quarter turns and a remainder |phi| <=
// pi/4, the remainder as lifting parameters (p, u) in float
template <int N, bool INV>
struct LiftTwiddles {
  int k[N];
  bool rest[N];
  float p[N];
  float u[N];
  constexpr LiftTwiddles() : k(), rest(), p(), u() {
    for (int j = 0; j < N; ++j) {
      const long num = INV ? 4L * j : -4L * j;          // angle in quarter turns, times N
      long kq = (num >= 0) ? (num + N / 2) / N : -((-num + N / 2) / N);
      const long m = num - kq * N;                        // remainder angle = 2 pi m / (4N)
      k[j] = static_cast<int>(((kq % 4) + 4) % 4);
      rest[j] = (m != 0);
      double s = 0.0, c = 1.0;
      ct_sincos_frac(m, 4L * N, &s, &c);
      p[j] = static_cast<float>(-s / (1.0 + c));
      u[j] = static_cast<float>(s);
    }
  }
};

template <int N>
struct Twiddles {
  double c[N];
  double s[N];
  constexpr Twiddles() : c(), s() {
    for (int j = 0; j < N; ++j) {
      double ss = 0.0, cc = 0.0;
      ct_sincos_frac(j, N, &ss, &cc);
      c[j] = cc;
      s[j] = ss;
    }
  }
};

}  // namespace msqd
