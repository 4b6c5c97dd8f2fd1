// FP32 (complex64) instantiation of the fused molecular step, with the
// J<->angle transform on FP32 matrix cores.
#include "mol_impl.h"

namespace msqd {
int launch_mol_fp32(const MolArgs& a, int n_r, hipStream_t s) { return launch_mol_any<float, kCpExact>(a, n_r, s); }
}  // namespace msqd
