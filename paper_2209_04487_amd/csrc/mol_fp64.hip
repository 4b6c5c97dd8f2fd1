// FP64 (complex128) instantiation of the fused molecular step.
#include "mol_impl.h"

namespace msqd {
int launch_mol_fp64(const MolArgs& a, int n_r, hipStream_t s) { return launch_mol_any<double, kCpExact>(a, n_r, s); }
}  // namespace msqd
