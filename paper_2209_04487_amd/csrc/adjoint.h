// Adjoint (reverse-mode) kernels of the coupled step: launch arguments.
#pragma once

#include "fdtd.h"
#include "mol.h"

namespace msqd {

struct MolAdjArgs {
  int n_mol, nj, kdiss;
  double dr;
  const void* psi_n;      // state before the step (recomputed forward inside)
  void* psi_np1;          // state after the step (FP64: overwritten, scratch), or nullptr (then recomputed too)
  const double* E_mol;    // field used by the step (au)
  void* lpsi;             // in: adjoint after the step; out: before
  const double* labs;     // adjoint of the absorbed norm (unchanged by the step)
  const double* ld;       // adjoint of the dipole written by the step
  double* lE;             // out: adjoint of the gathered field (au)
  const char* ws;
  QdLayout lay;
};
int launch_mol_adj(const MolAdjArgs& a, int n_r, bool f32, hipStream_t s);
size_t mol_adj_lds_bytes(int n_r, int nj, bool f32);

struct FdAdjArgs {
  FdArgs f;                // coefficients, mat, and the adjoint field pointers in place of fields
  void* scratch;           // 6 x n cells, field element type
};
int launch_yee_e_adj(const FdAdjArgs& a, bool f32, hipStream_t s);

struct CplAdjArgs {
  int n_occ;
  double pfac, inv_dt, inv_eau;
  double ce[4];
  const int* occ_cell;
  const int* occ_ptr;
  const int* mol_perm;
  const uint8_t* mat;
  double* lP;
  double* ld;
  const double* lE;
  void* lEx;
  // multi-rate coupling (molecules every M field steps): the adjoint of the
  // held current per occupied cell, accumulated over the held steps; NULL
  // for M = 1.  update: this step recomputes P_c and the current;
  // inv_mdt = 1 / (M dt).
  double* lJ;
  int update;
  double inv_mdt;
};
// One launch: g = (2/(eta0 dx)) sum over the source plane of ce[mat]
// lambda_Ex, and the deposit's adjoint over dep.n_occ occupied cells (none
// when dep.n_occ is 0).  Both read lambda_Ex before the E update's adjoint.
int launch_src_grad_deposit_adj(const FdArgs& lam, double coef, double* g_out, const CplAdjArgs& dep, bool f32,
                                hipStream_t s);
// The H update's adjoint; the gather's adjoint over gat.n_occ occupied cells
// (none when 0) rides in its first launch, which touches no lambda_E.
int launch_yee_h_adj(const FdAdjArgs& a, const CplAdjArgs& gat, bool f32, hipStream_t s);

// lambda_psi = scale * 2 dr psi for r > r_diss, else 0; labs = scale
int launch_yield_adj_init(void* lpsi, double* labs, const void* psi, int n_mol, int lines, int n_r,
                          int kdiss, double dr, double scale, bool f32, hipStream_t s);

}  // namespace msqd
