// In-register DFTs of small power-of-two sizes, fully unrolled (radix-4
// decimation in time, one radix-2 stage when log2 N is odd), with the
// twiddle factors folded to constants at compile time: (cos, sin) products in
// double, lifting rotations in float.
#pragma once

#include "common.h"

namespace msqd {

template <int N>
__host__ __device__ __forceinline__ double tw_cos(int j) {
  constexpr Twiddles<N> t{};
  return t.c[j];
}
template <int N>
__host__ __device__ __forceinline__ double tw_sin(int j) {
  constexpr Twiddles<N> t{};
  return t.s[j];
}

// v * exp(-2 pi i j / N) (forward) or v * exp(+2 pi i j / N) (inverse)
template <int N, bool INV, typename T>
__host__ __device__ __forceinline__ cx<T> mul_tw(cx<T> v, int j) {
  j %= N;
  if (j == 0) return v;
  if ((4 * j) % N == 0) {
    const int q = (4 * j) / N;  // quarter turns
    if (q == 2) return {-v.x, -v.y};
    // forward: exp(-i pi/2 q); q = 1 -> -i, q = 3 -> +i
    const bool times_minus_i = (q == 1) != INV;
    return times_minus_i ? mul_mi(v) : mul_i(v);
  }
  if constexpr (sizeof(T) == 4) {
    // float: exact quarter turns, then the remainder by lifting (no
    // systematic modulus error; see lift_rot)
    constexpr LiftTwiddles<N, INV> L{};
    cx<T> w = v;
    switch (L.k[j]) {
      case 1: w = mul_i(w); break;
      case 2: w = cx<T>{-w.x, -w.y}; break;
      case 3: w = mul_mi(w); break;
      default: break;
    }
    return L.rest[j] ? lift_rot(w, L.p[j], L.u[j]) : w;
  } else {
    const T c = static_cast<T>(tw_cos<N>(j));
    const T s = INV ? static_cast<T>(tw_sin<N>(j)) : static_cast<T>(-tw_sin<N>(j));
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// In-place DFT of x[0..N-1]: X[k] = sum_n x[n] exp(-+2 pi i n k / N), no scaling.
template <int N, bool INV, typename T>
__host__ __device__ __forceinline__ void dft(cx<T>* x) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2) {
    const cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  } else if constexpr (N % 4 == 0) {
    constexpr int M = N / 4;
    cx<T> s0[M], s1[M], s2[M], s3[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      s0[m] = x[4 * m + 0];
      s1[m] = x[4 * m + 1];
      s2[m] = x[4 * m + 2];
      s3[m] = x[4 * m + 3];
    }
    dft<M, INV, T>(s0);
    dft<M, INV, T>(s1);
    dft<M, INV, T>(s2);
    dft<M, INV, T>(s3);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const cx<T> a0 = s0[k];
      const cx<T> a1 = mul_tw<N, INV, T>(s1[k], k);
      const cx<T> a2 = mul_tw<N, INV, T>(s2[k], 2 * k);
      const cx<T> a3 = mul_tw<N, INV, T>(s3[k], 3 * k);
      const cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
      x[k] = t0 + t2;
      x[k + 2 * M] = t0 - t2;
      if (!INV) {
        x[k + M] = t1 + mul_mi(t3);
        x[k + 3 * M] = t1 + mul_i(t3);
      } else {
        x[k + M] = t1 + mul_i(t3);
        x[k + 3 * M] = t1 + mul_mi(t3);
      }
    }
  } else {
    constexpr int M = N / 2;
    cx<T> e[M], o[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      e[m] = x[2 * m];
      o[m] = x[2 * m + 1];
    }
    dft<M, INV, T>(e);
    dft<M, INV, T>(o);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const cx<T> t = mul_tw<N, INV, T>(o[k], k);
      x[k] = e[k] + t;
      x[k + M] = e[k] - t;
    }
  }
}

}  // namespace msqd
