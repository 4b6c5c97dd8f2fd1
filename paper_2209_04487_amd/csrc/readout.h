// Excited-state radial moments (Eq. (8)) of the wavepackets.
#pragma once

#include "common.h"

namespace msqd {

struct RdArgs {
  int n_mol, nj, n_r;
  double r_min, dr;
  const void* psi;       // cx<T> [n_mol][2][nj][n_r]
  double* r_num;         // [n_mol]
  double* pop;           // [n_mol]
  double* sums;          // [2] or nullptr
};

int launch_excited_r(const RdArgs& a, bool f32, hipStream_t s);

}  // namespace msqd
