// FP32 (complex64) instantiation of the fused molecular step, with the
// J<->angle transform on the vector ALUs.
#include "mol_impl.h"

namespace msqd {
int launch_mol_fp32(const MolArgs& a, int n_r, hipStream_t s) { return launch_mol_any<float, false>(a, n_r, s); }
}  // namespace msqd
