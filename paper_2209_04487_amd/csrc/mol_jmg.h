// The rotational basis |j, m>, j <= j_max for j_max >= 2: the tables of the
// exact coupling exp(i mu12(r) dt sigma_x (x) A), A = sum_c E_c D_c (Eq. (3)
// with the X, Y, Z direction cosines of the molecular axis).
//
// With |E| = e and the field direction at polar angle beta and azimuth alpha,
// A = e U D_z U^H, where U is the rotation exp(-i alpha J_z) exp(-i beta J_y)
// in the |j, m> basis (block diagonal in j, U[(j,m),(j,m')] =
// exp(-i m alpha) d^j_{m m'}(beta)) and D_z the direction cosine along z,
// which keeps m and is tridiagonal in j.  Each m' block of D_z is
// diagonalised once on the host, D_z|m' = Q diag(x) Q^T, so that the coupling
// at a radial point is: rotate to the field frame (U^H), transform each m'
// block to the eigenbasis of cos(theta) (Q^T), rotate the (g, e) pair of every
// eigenvector by the angle mu12(r) dt e x_k, and transform back.  The Wigner
// matrices d^j(beta) are formed per molecule from the eigenvectors of J_x:
// exp(-i beta J_y) = exp(-i pi/2 J_z) exp(-i beta J_x) exp(i pi/2 J_z), so
//   d^j_{m m'}(beta) = sum_k O_{m k} O_{m' k} cos(pi/2 (m' - m) - beta mu_k),
// J_x = O diag(mu) O^T with mu_k = k - j.
//
// The tables sit in the qd workspace after the common tables (at
// QdLayout::total), as doubles:
//   jx  : O^(j) for j = 0..j_max, (2j+1)^2 each, row m + j, column k
//         (eigenvalue k - j);
//   q   : Q^(a) for a = |m'| = 0..j_max, (j_max+1-a)^2 each, row j - a,
//         column k (ascending eigenvalues);
//   x   : the eigenvalues x^(a)_k, j_max+1-a each;
//   dip : per basis state b = j^2 + m + j: <j+1,m|cos th|j,m>,
//         <j+1,m+1|sin th e^{i ph}|j,m>, <j-1,m+1|sin th e^{i ph}|j,m> (the
//         matrix elements of the dipole readout; zero where the target state
//         is outside the basis).
#pragma once

#include <hip/hip_runtime.h>

#include "mol.h"

namespace msqd {

constexpr int kJmgMax = 5;   // largest j_max of the general (j, m) step

__host__ __device__ constexpr int jmg_nb(int jm) { return (jm + 1) * (jm + 1); }
// sum_{j' < j} (2j' + 1)^2
__host__ __device__ constexpr int jmg_jx_off(int j) { return j * (4 * j * j - 1) / 3; }
__host__ __device__ constexpr int jmg_sq_sum(int n) { return n * (n + 1) * (2 * n + 1) / 6; }
// sum_{a' < a} (jm + 1 - a')^2 and sum_{a' < a} (jm + 1 - a')
__host__ __device__ constexpr int jmg_q_off(int jm, int a) { return jmg_sq_sum(jm + 1) - jmg_sq_sum(jm + 1 - a); }
__host__ __device__ constexpr int jmg_x_off(int jm, int a) { return a * (jm + 1) - a * (a - 1) / 2; }

struct JmgTab {
  int jx, q, x, dip;   // offsets (doubles) of the four tables
  int n_jx, n_q, n_x;  // their lengths
  int n;               // total doubles
};
__host__ __device__ constexpr JmgTab jmg_tab(int jm) {
  const int n_jx = jmg_jx_off(jm + 1);
  const int n_q = jmg_q_off(jm, jm + 1);
  const int n_x = jmg_x_off(jm, jm + 1);
  return JmgTab{0, n_jx, n_jx + n_q, n_jx + n_q + n_x, n_jx, n_q, n_x, n_jx + n_q + n_x + 3 * jmg_nb(jm)};
}

// Host: fill the tables for j_max = jm (2 <= jm <= kJmgMax) into out[0 ..
// jmg_tab(jm).n).  Returns false if an eigen-decomposition fails to converge.
bool fill_jmg_tables(int jm, double* out);

// Host: whether the general (j, m) step is built for this grid, precision
// and j_max (at most 1024 threads and 160 KB of LDS per workgroup, the
// gfx950 limits); the LDS bytes of one workgroup go to *lds.  Needs no
// device.
bool jmg_supported(int n_r, bool f32, int jm, size_t* lds);

// Launch the general (j, m) step (returns a hipError_t value cast to int).
int launch_mol_jmg(const MolArgs& a, int n_r, bool f32, int jm, hipStream_t s);

}  // namespace msqd
