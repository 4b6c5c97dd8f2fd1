// General (j, m) molecular step, complex128 form.
#include <hip/hip_runtime.h>

#include "mol_jmg_impl.h"

namespace msqd {

int launch_mol_jmg_f64(const MolArgs& a, int n_r, int jm, hipStream_t s) {
  return launch_jmg_prec<double>(a, n_r, jm, s);
}

bool jmg_fits_f64(int n_r, int jm, size_t* lds) { return jmg_fits<double>(n_r, jm, lds); }

}  // namespace msqd
