// Readouts of the molecular state and the field monitor: the excited-state
// radial moments of Eq. (8), fixed-order FP64 ensemble sums of per-molecule
// values, and the T/R/A spectra from monitor fluxes.
#pragma once

#include "common.h"

namespace msqd {

struct RdArgs {
  int n_mol, nj, n_r;
  double r_min, dr;
  const void* psi;       // cx<T> [n_mol][2][nj][n_r]
  double* r_num;         // [n_mol]
  double* pop;           // [n_mol]
  double* sums;          // [3] or nullptr
};

int launch_excited_r(const RdArgs& a, bool f32, hipStream_t s);

// Ensemble sums: stage one reduces blocks of kSumBlock consecutive molecules
// to partials, stage two reduces the partials; the summation order depends
// only on n, so the result is bit-reproducible for a given batch size.
constexpr int kSumBlock = 1024;
constexpr int kMaxSumVecs = 5;   // three dipole components, norm, yield

inline int sum_blocks(int n) { return (n + kSumBlock - 1) / kSumBlock; }

struct SumArgs {
  const double* src[kMaxSumVecs];  // per-molecule values
  int stride[kMaxSumVecs];         // element stride of each (3 for one component of [n][3])
  int nv, n;
  double* partial;                 // [sum_blocks(n)][nv] scratch
  double* out;                     // [nv]
};

int launch_ensemble_sums(const SumArgs& a, hipStream_t s);

// T = S_trans / S_ref, R = (S_ref - S_inc) / S_ref, A = (S_inc - S_trans) / S_ref
int launch_spectra(const double* s_trans, const double* s_inc, const double* s_ref, int n_freq, double* tra,
                   hipStream_t s);

}  // namespace msqd
