// Molecular step: kernel arguments and the workspace layout of the tables.
#pragma once

#include <atomic>

#include "common.h"

namespace msqd {

constexpr int kMaxNJ = 16;

// With N_J <= 8 the exact-form contractions (16x16x4 matrix-core products)
// take two of the four K = 4 instructions: the J rows and angle nodes are
// placed in the operand positions those two read (FP64: rows 0-7 already;
// FP32: position 4g + i holds row 2g + i for i < 2, the FP32 fragment table
// is built in that order), the other positions are zero.
constexpr int kHalfKMaxNJ = 8;

// Tables in the qd workspace.  All offsets are bytes from the start of ws,
// each region 256-byte aligned.  The float64 tables feed the FP64 form, the
// float32 ones the FP32 / mixed forms; the bf16 blocks are the J<->angle
// matrix in matrix-core operand order (hi and lo parts).
struct QdLayout {
  size_t status;      // int32 flags (non-finite seen)
  size_t psi0;        // double [n_r] initial radial function
  size_t kin_d;       // cx<double> [n_r]  exp(-i k^2 dt / 4mu) / n_r, frequency order
  size_t tw_d;        // cx<double> [n_r]  exp(-2 pi i j / n_r)
  size_t vph_d;       // cx<double> [2][nj][n_r]
  size_t x_d;         // double [nj]      Gauss-Legendre nodes (ascending)
  size_t mudt_d;      // double [n_r]     mu12(r) dt
  size_t mask_d;      // double [n_r]
  size_t mu_d;        // double [n_r]     mu12(r) (readout)
  size_t cj_d;        // double [nj]      <J|cos|J+1>
  size_t kin_f, tw_f, vph_f, x_f, mudt_f, mask_f;   // float versions
  size_t tw_fs;       // cx<float> tw_f x n_r^(-1/2) when n_r is an even power of two (else tw_f)
  size_t tmfrag;      // bf16 matrix-core fragments of T and T^T (hi, lo)
  size_t tmfrag_d;    // double [2][64][4] matrix-core fragments of T and T^T
  size_t tmfrag_f;    // float  [2][64][4]
  size_t total;
};

QdLayout qd_layout(int n_r, int nj);

struct MolArgs {
  int n_mol;
  int nj;
  int n_steps;          // 0: readouts only, state untouched
  int kdiss;            // first radial index with r > r_diss
  int kmask;            // first radial index where the absorber mask is below one
  int want_d, want_norm, want_yield;
  double dr;
  void* psi;            // cx<T> [n_mol][2][nj][n_r]
  void* psi_out;        // where the stepped state goes (m = 0 kernels), or nullptr: back to psi
  const double* E_mol;  // [n_mol] field (au), used when Ex == nullptr
  const void* Ex;       // field array (double or float) or nullptr
  const void* Ey;       // (j, m) basis: the other two components, same cells
  const void* Ez;
  int ex_is_float;      // element type of Ex
  const int* cell_of_mol;
  double inv_eau;       // 1 / (V/m per au)
  double* E_out;        // [n_mol] field used (au), or nullptr
  double* absorbed;     // [n_mol]
  double* d_mol;        // [n_mol] or nullptr
  double* norm_mol;     // [n_mol] or nullptr
  double* yield_mol;    // [n_mol] or nullptr
  const char* ws;
  QdLayout lay;
  int* status;
};

// LDS bytes the fused step needs per workgroup, and the device's per-workgroup
// LDS limit (queried once).
size_t mol_lds_bytes(int n_r, int nj, int prec);
size_t mol_lds_limit();

// Let a kernel use more than 64 KB of dynamic LDS on the current device.  The
// attribute is per device: `done` keeps one bit per device id already set
// (ids >= 64 are set on every call).  Safe to call from several host threads.
hipError_t allow_large_lds(const void* kernel, std::atomic<unsigned long long>& done);

// launchers (return a hipError_t value cast to int)
int launch_mol_fp64(const MolArgs& a, int n_r, hipStream_t s);
// the (j, m)-basis step (j <= 1, three field components)
int launch_mol_jm(const MolArgs& a, int n_r, bool f32, hipStream_t s);
int launch_mol_fp32(const MolArgs& a, int n_r, hipStream_t s);
int launch_mol_mixed(const MolArgs& a, int n_r, hipStream_t s);

}  // namespace msqd
