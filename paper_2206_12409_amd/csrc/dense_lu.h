// Dense complex FP64 LU with partial pivoting on the device (dense_lu.hip).
#pragma once
#include "kernels.h"

namespace vsie {

// DenseLU (the factors and their device buffers) is declared in vsie_internal.h.
inline int64_t lu_blocks_elems(int n) { return (int64_t)((n + LU_NB - 1) / LU_NB) * LU_NB * LU_NB; }
int64_t lu_work_elems(int n);   // scratch of lu_factor

constexpr int LU_PERM_LDS = 8192;   // largest n whose pivot permutation is formed on the device

// Factor F.A in place; blocks on the stream at the end. Throws Error(VSIE_E_SINGULAR) for an
// exactly zero pivot column. The row permutation F.d_perm is formed on the host from the pivots
// read back (F.perm keeps a copy), or with device_perm on the device (n <= LU_PERM_LDS; F.perm
// stays empty and nothing is allocated on the host).
void lu_factor(hipStream_t st, DenseLU& F, cxd* work, bool device_perm = false);
// B (n x nrhs, row stride ldb) <- A^-1 B; W: n x nrhs scratch. Asynchronous.
void lu_solve(hipStream_t st, const DenseLU& F, cxd* B, int64_t ldb, int nrhs, cxd* W);

}  // namespace vsie
