// Frozen two-level (Bloch) emitters: RK4 kernel and launcher.
#pragma once

#include "common.h"

namespace msqd {

struct BlochArgs {
  int n;
  int n_steps;
  double w0, mu, g1, g2, dt;      // atomic units
  void* state;                    // T [3][n]: rho_ee, Re rho_ge, Im rho_ge
  const double* E;                // [n] field (au), used when Ex == nullptr
  const void* Ex;                 // field array (float or double) or nullptr
  int ex_is_float;
  const int* cell_of_mol;
  double inv_eau;
  double* E_out;                  // [n] field used, or nullptr
  double* d;                      // [n] dipole 2 mu Re rho_ge, or nullptr
};

int launch_bloch(const BlochArgs& a, bool f32, hipStream_t s);

}  // namespace msqd
