// Dense complex FP64 LU with partial pivoting on the device (dense_lu.hip).
#pragma once
#include "kernels.h"

namespace vsie {

// DenseLU (the factors and their device buffers) is declared in vsie_internal.h.
inline int64_t lu_blocks_elems(int n) { return (int64_t)((n + LU_NB - 1) / LU_NB) * LU_NB * LU_NB; }
int64_t lu_work_elems(int n);   // scratch of lu_factor

// Factor F.A in place; blocks on the stream at the end (reads the pivots back). Throws
// Error(VSIE_E_SINGULAR) for an exactly zero pivot column.
void lu_factor(hipStream_t st, DenseLU& F, cxd* work);
// B (n x nrhs, row stride ldb) <- A^-1 B; W: n x nrhs scratch. Asynchronous.
void lu_solve(hipStream_t st, const DenseLU& F, cxd* B, int64_t ldb, int nrhs, cxd* W);

}  // namespace vsie
