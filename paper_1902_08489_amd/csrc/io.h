// States from dense vectors and checkpoint files of states.
#pragma once

#include "engine.h"

namespace tdmps {

// Sequential-SVD MPS of a dense 4^L vector (interleaved complex, Fock order, zero outside the
// total charge Q), truncated to Dmax and the relative cut-off (Methods, Eq. (mps)); L <= 12.
Mps* mps_from_dense(Contractor& C, int L, Charge Q, const double* coeffs, int Dmax, double cutoff);
// Binary checkpoint: magic, L and total charge, the sector tables of all bonds, the site
// tensors in the panel layout (FP64 interleaved complex), an FNV-1a checksum of all of it.
void mps_save(const Mps* m, const char* path);
Mps* mps_load(Ctx* ctx, const char* path);

}  // namespace tdmps
