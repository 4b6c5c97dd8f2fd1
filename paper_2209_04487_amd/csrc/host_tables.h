// Host-side table and map builders.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include "common.h"

namespace msqd {

struct MolTablesHost {
  double dr = 0.0;
  int kdiss = 0;
  std::vector<std::complex<double>> kin, tw, tw_f, vph;
  std::vector<double> tm, x, mudt, mask, mu, cj;
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// radix of the first in-register FFT pass for a radial grid of n_r points
// and complex elements of el_bytes/2 per part
constexpr int fft_r1(int n_r, int el_bytes) {
  return n_r == 64 ? 8 : (n_r == 128 ? 16 : (n_r == 256 ? (el_bytes == 4 ? 32 : 16) : 32));
}
MolTablesHost build_mol_tables(const qd_desc& d, const double* U_g, const double* U_e,
                               const double* mu12);

// Lifting parameters (p, u) = (-tan(phi/2), sin phi) of the unit phase
// c + i s = exp(i phi), phi in (-pi, pi].
void lift_params(double c, double s, float* p, float* u);
// Float pair (cf, sf) for the unit number c + i s whose modulus is as close
// to one as the float grid allows: the larger component rounded to nearest,
// the smaller one the float nearest sqrt(1 - larger^2) (the phase moves by at
// most about 1e-6 rad for the angles of the transform tables).
void unit_pair_f32(double c, double s, float* cf, float* sf);

void place_slab(int32_t n_mol, int32_t nx, int32_t ny, uint64_t seed, int32_t k0, int32_t nk,
                int32_t* cell_of_mol);
int32_t build_csr(int32_t n_mol, int32_t n_cells, const int32_t* cell_of_mol, int32_t* occ_cell,
                  int32_t* occ_ptr, int32_t* mol_perm);

}  // namespace msqd

namespace msqd {
// J<->angle matrix in matrix-core operand order, bf16 hi and lo parts
// (used by the mixed-precision molecular step).
void fill_mfma_fragments(unsigned char* dst, const std::vector<double>& tm, int nj);
}  // namespace msqd
