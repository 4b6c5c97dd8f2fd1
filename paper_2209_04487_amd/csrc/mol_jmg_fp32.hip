// General (j, m) molecular step, complex64 forms (FP32 and mixed), and the
// dispatch over both precisions.
#include <hip/hip_runtime.h>

#include "mol_jmg_impl.h"

namespace msqd {

int launch_mol_jmg_f64(const MolArgs& a, int n_r, int jm, hipStream_t s);
bool jmg_fits_f64(int n_r, int jm, size_t* lds);

int launch_mol_jmg(const MolArgs& a, int n_r, bool f32, int jm, hipStream_t s) {
  return f32 ? launch_jmg_prec<float>(a, n_r, jm, s) : launch_mol_jmg_f64(a, n_r, jm, s);
}

bool jmg_supported(int n_r, bool f32, int jm, size_t* lds) {
  size_t b = 0;
  const bool ok = f32 ? jmg_fits<float>(n_r, jm, &b) : jmg_fits_f64(n_r, jm, &b);
  if (lds) *lds = b;
  return ok;   // the launch also checks the device's own per-workgroup LDS limit
}

}  // namespace msqd
