// Field solver: workspace layout and launchers.
#pragma once

#include "common.h"

namespace msqd {

struct FdLayout {
  size_t bE, aE, kE, bH, aH, kH;      // double [nz] CPML profiles (kE, kH hold 1/kappa)
  size_t bEf, aEf, kEf, bHf, aHf, kHf; // float [nz]
  size_t freqs;                        // double [n_freq]
  size_t total;
};
FdLayout fd_layout(const fdtd_desc* d);

struct FdArgs {
  int nx, ny, nz, npml, metal_id, src_k;
  double inv_dx, cH;                   // 1/dx, dt/mu0
  double ce[4];                        // dt/(eps0 eps_r[m])
  double alpha_d, beta_d;              // Drude recurrence
  double src_term;                     // -2 E_inc / (eta0 dx) on plane src_k (0: none)
  void *Ex, *Ey, *Ez, *Hx, *Hy, *Hz, *JDx, *JDy, *JDz, *psi;
  const uint8_t* mat;
  const char* ws;
  FdLayout lay;
  // held molecular current (coupled step): E update subtracts held[c] on
  // planes held_k0 .. held_k0 + held_nk - 1 for components c < held_nc
  const void* held;
  int held_k0, held_nk, held_nc;       // held_nc = 0: none
};

int launch_yee_h(const FdArgs& a, bool f32, hipStream_t s);
int launch_yee_e(const FdArgs& a, bool f32, hipStream_t s);

// samples staged behind the accumulators before one pass folds them in
constexpr int kMonRing = 8;

struct MonArgs {
  int nx, ny, mon_k, n_freq;
  double tE, tH, wdt;                  // sample times, weight (every * dt)
  const void *Ex, *Ey, *Hx, *Hy;
  double* dft;
  const double* freqs;
  double* ring;                        // [kMonRing][4][ny][nx] staged samples of this plane
  int slot;                            // stage: the slot written
  int ns;                              // fold: the samples staged, in time order
  double tEs[kMonRing], tHs[kMonRing]; // fold: their sample times
};
// one sample straight into the accumulators
int launch_monitor(const MonArgs& a, bool f32, hipStream_t s);
// one sample into ring slot a.slot
int launch_monitor_stage(const MonArgs& a, bool f32, hipStream_t s);
// the a.ns staged samples into the accumulators, in order (the same
// accumulator updates, in the same order, as a.ns direct samples)
int launch_monitor_fold(const MonArgs& a, hipStream_t s);
int launch_flux(int nx, int ny, int n_freq, const double* dft, double* flux, hipStream_t s);

struct DepArgs {
  int n_occ;
  int update;                          // 1: new P from the dipoles; 0: apply the held J_mol
  double pfac;                         // w e a0 / dx^3
  double inv_dt;
  double ce[4];
  const double* d_mol;
  const int* occ_cell;
  const int* occ_ptr;
  const int* mol_perm;
  const uint8_t* mat;                  // E_x material ids
  double* P_c;                         // [n_occ][ncomp]
  double* J_mol;                       // [n_occ][ncomp]
  void* Ex;
  int ncomp;                           // 1: E_x only; 3: E_x, E_y, E_z (d_mol [n][3])
  void *Ey, *Ez;
  long ncells;                         // cells per component array (material planes)
  // non-null: write dt/(eps0 eps_r) J into held ([ncomp][held_nk][plane])
  // instead of subtracting it from E
  void* held;
  int held_k0, held_nk;
  long plane;                          // nx ny
};
int launch_deposit(const DepArgs& a, bool f32, hipStream_t s);

int launch_fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace msqd
