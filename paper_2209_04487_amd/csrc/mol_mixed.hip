// Mixed-precision instantiation of the fused molecular step: complex64
// wavepackets and FFTs, the J<->angle transform on BF16 matrix cores.
#include <cmath>
#include <cstring>
#include <vector>

#include "host_tables.h"
#include "mol_impl.h"

namespace msqd {

int launch_mol_mixed(const MolArgs& a, int n_r, hipStream_t s) {
  return launch_mol_any<float, kCpBf16x3>(a, n_r, s);
}

namespace {
unsigned short host_bf16_rne(float x) {
  unsigned int u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
float host_bf16_val(unsigned short b) {
  const unsigned int u = static_cast<unsigned int>(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
}  // namespace

// Operand fragments of the 16x16x16 matrix-core product: lane l supplies
// A[l % 16][4 (l / 16) + i], i = 0..3.  Block 0/1: A = T (rows = nodes,
// columns = J), hi/lo; block 2/3: A = T^T, hi/lo.  Entries outside nj are 0.
void fill_mfma_fragments(unsigned char* dst, const std::vector<double>& tm, int nj) {
  unsigned short* out = reinterpret_cast<unsigned short*>(dst);
  for (int lane = 0; lane < 64; ++lane) {
    for (int i = 0; i < 4; ++i) {
      const int row = lane % 16, colk = 4 * (lane / 16) + i;
      const double t = (row < nj && colk < nj) ? tm[static_cast<size_t>(row) * nj + colk] : 0.0;
      const double tt = (row < nj && colk < nj) ? tm[static_cast<size_t>(colk) * nj + row] : 0.0;
      const float tf = static_cast<float>(t), ttf = static_cast<float>(tt);
      const unsigned short th = host_bf16_rne(tf), tth = host_bf16_rne(ttf);
      out[(0 * 64 + lane) * 4 + i] = th;
      out[(1 * 64 + lane) * 4 + i] = host_bf16_rne(tf - host_bf16_val(th));
      out[(2 * 64 + lane) * 4 + i] = tth;
      out[(3 * 64 + lane) * 4 + i] = host_bf16_rne(ttf - host_bf16_val(tth));
    }
  }
}

}  // namespace msqd
