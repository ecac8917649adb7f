// Dense complex FP64 LU factorisation with partial pivoting, P A = L U, and solves with many
// right-hand sides, for row-major matrices resident in HBM.
//
// Used to eliminate the far-conductor unknowns from the coupled system (the Schur complement of
// the dense far block, the elimination the paper's conclusion proposes) and to invert the
// near-coil block that preconditions the reduced system.
//
// Right-looking blocked algorithm with panels of LU_NB columns:
//   1. panel: for each column j, pivot search over rows j.. (|re| + |im|, ties to the lowest row),
//      interchange of the two rows inside the panel, then one wavefront per row below scales the
//      multiplier and applies the rank-one update to the rest of the panel row;
//   2. the panel's interchanges are applied to the columns left and right of it;
//   3. the diagonal block's unit-lower and upper triangles are inverted (one workgroup, kept for
//      the solves), U12 = L11^-1 A12 is one matrix-core GEMM;
//   4. trailing update A22 -= L21 U12 on the matrix cores (k_zgemm_mfma, negated accumulation).
// Solves gather the rows by the pivot permutation and run block forward and back substitution
// with the inverted diagonal blocks, each block step a pair of GEMMs.
#include "dense_lu.h"

namespace vsie {

// pivot of column j: row p >= j maximising |re| + |im|; rows j and p swapped inside the panel
// columns [k, kend). One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_lu_pivot(cxd* __restrict__ A, int64_t lda, int n, int j, int k, int kend,
                                                   int* __restrict__ ipiv, int* __restrict__ info) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  double best = -1;
  int bidx = n;
  for (int i = j + threadIdx.x; i < n; i += 1024) {
    const cxd a = A[(int64_t)i * lda + j];
    const double v = fabs(a.re) + fabs(a.im);
    if (v > best) {
      best = v;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = bv[threadIdx.x + s];
      const int oi = bi[threadIdx.x + s];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int p = bi[0];
  if (threadIdx.x == 0) {
    ipiv[j] = p;
    if (!(bv[0] > 0) && *info == 0) *info = j + 1;   // exactly singular (or NaN) column
  }
  if (p != j && p < n) {
    for (int c = k + (int)threadIdx.x; c < kend; c += 1024) {
      const cxd t = A[(int64_t)j * lda + c];
      A[(int64_t)j * lda + c] = A[(int64_t)p * lda + c];
      A[(int64_t)p * lda + c] = t;
    }
  }
}

// rows i > j: l = A[i][j] / A[j][j], A[i][j] = l, A[i][c] -= l A[j][c] for panel columns c in
// (j, kend). One wavefront per row, lane = column offset; 4 rows per workgroup.
__global__ __launch_bounds__(256) void k_lu_rank1(cxd* __restrict__ A, int64_t lda, int n, int j, int kend) {
  const int i = j + 1 + blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (i >= n) return;
  const cxd piv = A[(int64_t)j * lda + j];
  if (piv.re == 0 && piv.im == 0) return;   // singular column, reported through info
  const cxd l = A[(int64_t)i * lda + j] * cinv(piv);
  const int c = j + 1 + lane;
  if (c < kend) A[(int64_t)i * lda + c] -= l * A[(int64_t)j * lda + c];
  if (lane == 0) A[(int64_t)i * lda + j] = l;
}

// apply the interchanges j <-> ipiv[j], j in [k, kend), to every column outside [k, kend)
__global__ void k_lu_laswp(cxd* __restrict__ A, int64_t lda, int n, int k, int kend, const int* __restrict__ ipiv) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int width = kend - k;
  if (c >= n - width) return;
  if (c >= k) c += width;
  for (int j = k; j < kend; ++j) {
    const int p = ipiv[j];
    if (p == j || p < 0 || p >= n) continue;   // p == n marks a NaN column (reported through info)
    const cxd t = A[(int64_t)j * lda + c];
    A[(int64_t)j * lda + c] = A[(int64_t)p * lda + c];
    A[(int64_t)p * lda + c] = t;
  }
}

// inverses of the unit-lower and the upper triangle of the nb x nb diagonal block at (k, k):
// threads 0..nb-1 build the columns of L^-1, threads 64..64+nb-1 those of U^-1 (row-major,
// leading dimension LU_NB). The block is staged in LDS; each thread writes only its own column.
__global__ __launch_bounds__(128) void k_lu_tri_inv(const cxd* __restrict__ A, int64_t lda, int k, int nb,
                                                    cxd* __restrict__ Linv, cxd* __restrict__ Uinv) {
  __shared__ cxd D[LU_NB][LU_NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 128) D[e / nb][e % nb] = A[(int64_t)(k + e / nb) * lda + k + e % nb];
  __syncthreads();
  const int c = threadIdx.x % 64;
  if (c >= nb) return;
  if (threadIdx.x < 64) {
    // column c of L^-1: x_r = 0 (r < c), x_c = 1, x_r = -sum_{c <= s < r} L[r][s] x_s
    for (int r = 0; r < nb; ++r) {
      cxd x = {r == c ? 1.0 : 0.0, 0.0};
      if (r > c) {
        cxd s = {0, 0};
        for (int q = c; q < r; ++q) s += D[r][q] * Linv[q * LU_NB + c];
        x = cxd{-s.re, -s.im};
      }
      Linv[r * LU_NB + c] = x;
    }
  } else {
    // column c of U^-1: x_r = 0 (r > c), x_c = 1 / U[c][c], x_r = -(sum_{r < s <= c} U[r][s] x_s) / U[r][r]
    for (int r = nb - 1; r >= 0; --r) {
      cxd x = {0, 0};
      if (r == c) {
        x = cinv(D[c][c]);
      } else if (r < c) {
        cxd s = {0, 0};
        for (int q = r + 1; q <= c; ++q) s += D[r][q] * Uinv[q * LU_NB + c];
        x = cxd{-s.re, -s.im} * cinv(D[r][r]);
      }
      Uinv[r * LU_NB + c] = x;
    }
  }
}

// dst[r][c] = src[r][c] for an r x c block (row strides ls, ld)
__global__ void k_copy2d(const cxd* __restrict__ src, int64_t ls, cxd* __restrict__ dst, int64_t ld, int rows,
                         int cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  dst[r * ld + c] = src[r * ls + c];
}

// dst[i][:] = src[perm[i]][:]
__global__ void k_gather_rows(const cxd* __restrict__ src, int64_t ls, const int* __restrict__ perm,
                              cxd* __restrict__ dst, int64_t ld, int rows, int cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  dst[r * ld + c] = src[(int64_t)perm[r] * ls + c];
}

static unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// C = (negate ? -1 : 1) A B (+ C when accumulate), all row-major with the given row strides
static void gemm_rm(hipStream_t st, int M, int N, int K, const cxd* A, int64_t lda, const cxd* B, int64_t ldb, cxd* C,
                    int64_t ldc, int accumulate, int negate) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  GemmSet<double> S{};
  S.nprob = 1;
  S.nbatch[0] = 1;
  GemmArgs<double>& g = S.g[0];
  g.A = A;
  g.sar = lda;
  g.sac = 1;
  g.B = B;
  g.sbr = ldb;
  g.sbc = 1;
  g.C = C;
  g.scr = ldc;
  g.scc = 1;
  g.M = M;
  g.N = N;
  g.K = K;
  g.accumulate = accumulate;
  g.negate = negate;
  launch_zgemm<double>(st, S);
}

int64_t lu_work_elems(int n) { return (int64_t)LU_NB * std::max(n, 1); }

void lu_factor(hipStream_t st, DenseLU& F, cxd* work) {
  const int n = F.n;
  const int64_t lda = F.lda;
  cxd* A = F.A;
  VSIE_HIP(hipMemsetAsync(F.d_info, 0, sizeof(int), st));
  for (int k = 0, p = 0; k < n; k += LU_NB, ++p) {
    const int nb = std::min(LU_NB, n - k);
    const int kend = k + nb;
    for (int j = k; j < kend; ++j) {
      hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(1024), 0, st, A, lda, n, j, k, kend, F.d_ipiv, F.d_info);
      if (j + 1 < n) hipLaunchKernelGGL(k_lu_rank1, dim3(nblocks(n - j - 1, 4)), dim3(256), 0, st, A, lda, n, j, kend);
    }
    if (n > nb) hipLaunchKernelGGL(k_lu_laswp, dim3(nblocks(n - nb, 256)), dim3(256), 0, st, A, lda, n, k, kend, F.d_ipiv);
    cxd* Li = F.Linv + (int64_t)p * LU_NB * LU_NB;
    cxd* Ui = F.Uinv + (int64_t)p * LU_NB * LU_NB;
    hipLaunchKernelGGL(k_lu_tri_inv, dim3(1), dim3(128), 0, st, A, lda, k, nb, Li, Ui);
    const int nr = n - kend;
    if (nr > 0) {
      // U12 = L11^-1 A12 (A12 copied out first), then A22 -= L21 U12
      hipLaunchKernelGGL(k_copy2d, dim3(nblocks((int64_t)nb * nr, 256)), dim3(256), 0, st, A + (int64_t)k * lda + kend,
                         lda, work, (int64_t)nr, nb, nr);
      gemm_rm(st, nb, nr, nb, Li, LU_NB, work, nr, A + (int64_t)k * lda + kend, lda, 0, 0);
      gemm_rm(st, nr, nr, nb, A + (int64_t)kend * lda + k, lda, A + (int64_t)k * lda + kend, lda,
              A + (int64_t)kend * lda + kend, lda, 1, 1);
    }
  }
  VSIE_HIP(hipGetLastError());
  std::vector<int> ipiv(n);
  int info = 0;
  if (n > 0) VSIE_HIP(hipMemcpyAsync(ipiv.data(), F.d_ipiv, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  VSIE_HIP(hipMemcpyAsync(&info, F.d_info, sizeof(int), hipMemcpyDeviceToHost, st));
  VSIE_HIP(hipStreamSynchronize(st));
  if (info != 0)
    throw Error(VSIE_E_SINGULAR, "dense LU: exactly singular pivot in column " + std::to_string(info - 1));
  // row permutation: the interchanges applied in order to the identity
  F.perm.resize(n);
  for (int i = 0; i < n; ++i) F.perm[i] = i;
  for (int j = 0; j < n; ++j) std::swap(F.perm[j], F.perm[ipiv[j]]);
  if (n > 0) {
    VSIE_HIP(hipMemcpyAsync(F.d_perm, F.perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    VSIE_HIP(hipStreamSynchronize(st));
  }
}

void lu_solve(hipStream_t st, const DenseLU& F, cxd* B, int64_t ldb, int nrhs, cxd* W) {
  const int n = F.n;
  const int64_t lda = F.lda;
  if (n <= 0 || nrhs <= 0) return;
  const int64_t ldw = nrhs;
  // W = P B; forward substitution writes Y into B, back substitution X into W
  hipLaunchKernelGGL(k_gather_rows, dim3(nblocks((int64_t)n * nrhs, 256)), dim3(256), 0, st, B, ldb, F.d_perm, W, ldw,
                     n, nrhs);
  const int np = (n + LU_NB - 1) / LU_NB;
  for (int p = 0; p < np; ++p) {
    const int k = p * LU_NB, nb = std::min(LU_NB, n - k), kend = k + nb;
    gemm_rm(st, nb, nrhs, nb, F.Linv + (int64_t)p * LU_NB * LU_NB, LU_NB, W + k * ldw, ldw, B + k * ldb, ldb, 0, 0);
    gemm_rm(st, n - kend, nrhs, nb, F.A + (int64_t)kend * lda + k, lda, B + k * ldb, ldb, W + kend * ldw, ldw, 1, 1);
  }
  for (int p = np - 1; p >= 0; --p) {
    const int k = p * LU_NB, nb = std::min(LU_NB, n - k);
    gemm_rm(st, nb, nrhs, nb, F.Uinv + (int64_t)p * LU_NB * LU_NB, LU_NB, B + k * ldb, ldb, W + k * ldw, ldw, 0, 0);
    gemm_rm(st, k, nrhs, nb, F.A + k, lda, W + k * ldw, ldw, B, ldb, 1, 1);
  }
  hipLaunchKernelGGL(k_copy2d, dim3(nblocks((int64_t)n * nrhs, 256)), dim3(256), 0, st, W, ldw, B, ldb, n, nrhs);
  VSIE_HIP(hipGetLastError());
}

}  // namespace vsie
