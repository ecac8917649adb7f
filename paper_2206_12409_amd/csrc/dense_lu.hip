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
//      multiplier and applies the rank-one update to the rest of the panel row; the update also
//      reduces the next column's pivot candidates per workgroup, so only a panel's first column
//      is searched by reading it;
//   2. the panel's interchanges are applied to the columns left and right of it;
//   3. the diagonal block's unit-lower and upper triangles are inverted (one workgroup, kept for
//      the solves); the panel's U rows to its right are L11^-1 times those rows once the U rows
//      of the group's earlier panels have been taken out of them (two matrix-core GEMMs);
//   4. trailing update A22 -= L21 U12 on the matrix cores (k_zgemm_mfma, negated accumulation),
//      taken once per group of LU_GROUP panels (depth LU_GROUP LU_NB); inside a group each panel is
//      first updated by the group's earlier panels alone.
// Solves gather the rows by the pivot permutation and run block forward and back substitution
// with the inverted diagonal blocks, each block step a pair of GEMMs.
#include "dense_lu.h"

namespace vsie {

// (best, bidx) of every thread of a 1024-thread workgroup reduced to the largest |re| + |im|, lowest
// row among ties; then ipiv[j] = p, info set on an exactly zero (or NaN) column, rows j and p
// swapped inside the panel columns [k, kend)
__device__ void pivot_reduce_finish(double best, int bidx, cxd* __restrict__ A, int64_t lda, int n, int j, int k,
                                    int kend, int* __restrict__ ipiv, int* __restrict__ info) {
  __shared__ double bv[16];
  __shared__ int bi[16];
  auto combine = [&](double o, int oi) {
    if (o > best || (o == best && oi < bidx)) {
      best = o;
      bidx = oi;
    }
  };
  for (int off = 32; off > 0; off >>= 1) combine(__shfl_xor(best, off), __shfl_xor(bidx, off));
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    bv[wave] = best;
    bi[wave] = bidx;
  }
  __syncthreads();
  if (wave == 0) {
    best = lane < 16 ? bv[lane] : -1;
    bidx = lane < 16 ? bi[lane] : n;
    for (int off = 8; off > 0; off >>= 1) combine(__shfl_xor(best, off), __shfl_xor(bidx, off));
    if (lane == 0) {
      bv[0] = best;
      bi[0] = bidx;
    }
  }
  __syncthreads();
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

// pivot of the first column j of a panel: row p >= j maximising |re| + |im|, found by reading the
// column; rows j and p swapped inside the panel columns [k, kend). One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_lu_pivot(cxd* __restrict__ A, int64_t lda, int n, int j, int k, int kend,
                                                   int* __restrict__ ipiv, int* __restrict__ info) {
  double best = -1;
  int bidx = n;
  // eight independent loads in flight per thread; within a thread rows increase, so the strict
  // comparison keeps the lowest row among equal magnitudes (NaN never wins)
  constexpr int U = 8;
  for (int i0 = j + (int)threadIdx.x; i0 < n; i0 += 1024 * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 1024 * u;
      v[u] = -1;
      if (i < n) {
        const cxd a = A[(int64_t)i * lda + j];
        v[u] = fabs(a.re) + fabs(a.im);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v[u] > best) {
        best = v[u];
        bidx = i0 + 1024 * u;
      }
  }
  pivot_reduce_finish(best, bidx, A, lda, n, j, k, kend, ipiv, info);
}

// pivot of the other columns of a panel, from the nparts candidates the rank-one update of column
// j - 1 left (one per workgroup, in row order): the same choice as k_lu_pivot without reading
// a column of the matrix (one row per page at these leading dimensions).
__global__ __launch_bounds__(1024) void k_lu_pivot_parts(cxd* __restrict__ A, int64_t lda, int n, int j, int k,
                                                         int kend, const double* __restrict__ pv,
                                                         const int* __restrict__ pi, int nparts,
                                                         int* __restrict__ ipiv, int* __restrict__ info) {
  double best = -1;
  int bidx = n;
  constexpr int U = 4;
  for (int b0 = (int)threadIdx.x; b0 < nparts; b0 += 1024 * U) {
    double v[U];
    int r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + 1024 * u;
      v[u] = b < nparts ? pv[b] : -1;
      r[u] = b < nparts ? pi[b] : n;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (v[u] > best) {
        best = v[u];
        bidx = r[u];
      }
  }
  pivot_reduce_finish(best, bidx, A, lda, n, j, k, kend, ipiv, info);
}

// rows i > j: l = A[i][j] / A[j][j], A[i][j] = l, A[i][c] -= l A[j][c] for panel columns c in
// (j, kend). One wavefront per row, lane = column offset; 4 rows per workgroup. With pv given, each
// workgroup also leaves the pivot candidate of column j + 1 among its rows (largest |re| + |im| of
// the updated entries, lowest row among ties, NaN never chosen) in pv/pi[blockIdx.x].
__global__ __launch_bounds__(256) void k_lu_rank1(cxd* __restrict__ A, int64_t lda, int n, int j, int kend,
                                                  double* __restrict__ pv, int* __restrict__ pi) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = j + 1 + blockIdx.x * 4 + w;
  const int c = j + 1 + lane;
  double v = -1;
  if (i < n) {
    const cxd piv = A[(int64_t)j * lda + j];
    if (piv.re != 0 || piv.im != 0) {
      const cxd l = A[(int64_t)i * lda + j] * cinv(piv);
      if (c < kend) {
        const cxd t = A[(int64_t)i * lda + c] - l * A[(int64_t)j * lda + c];
        A[(int64_t)i * lda + c] = t;
        v = fabs(t.re) + fabs(t.im);
      }
      if (lane == 0) A[(int64_t)i * lda + j] = l;
    } else if (c < kend) {   // singular column, reported through info: entries left as they are
      const cxd t = A[(int64_t)i * lda + c];
      v = fabs(t.re) + fabs(t.im);
    }
  }
  if (!pv) return;
  if (lane == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double best = -1;
    int bidx = n;
    for (int q = 0; q < 4; ++q)
      if (sv[q] > best) {
        best = sv[q];
        bidx = si[q];
      }
    pv[blockIdx.x] = best;
    pi[blockIdx.x] = bidx;
  }
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

// inverses of the unit-lower and the upper triangle of the nb x nb diagonal block at (k, k) (row-major,
// leading dimension LU_NB). The block is staged in LDS; one wavefront per column of L^-1 or U^-1
// (16 wavefronts, 8 columns each), lane r holding entry r: the substitution runs column by column
// of the triangle, each finished entry broadcast across the wavefront and eliminated from the rows
// still open.
__global__ __launch_bounds__(1024) void k_lu_tri_inv(const cxd* __restrict__ A, int64_t lda, int k, int nb,
                                                     cxd* __restrict__ Linv, cxd* __restrict__ Uinv) {
  __shared__ cxd D[LU_NB][LU_NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 1024) D[e / nb][e % nb] = A[(int64_t)(k + e / nb) * lda + k + e % nb];
  __syncthreads();
  const int wave = threadIdx.x / 64, r = threadIdx.x % 64;
  for (int g = wave; g < 2 * LU_NB; g += 16) {
    const bool lower = g < LU_NB;
    const int c = lower ? g : g - LU_NB;
    if (c >= nb) continue;
    cxd x = {r == c ? 1.0 : 0.0, 0.0};
    if (lower) {
      // L x = e_c: x_s final at step s, then x_r -= L[r][s] x_s for r > s
      for (int s = c; s + 1 < nb; ++s) {
        const cxd xs = {__shfl(x.re, s), __shfl(x.im, s)};
        if (r > s && r < nb) x -= D[r][s] * xs;
      }
      if (r < nb) Linv[r * LU_NB + c] = x;
    } else {
      // U x = e_c, from the bottom: x_s /= U[s][s] at step s, then x_r -= U[r][s] x_s for r < s
      for (int s = c; s >= 0; --s) {
        if (r == s) x = x * cinv(D[s][s]);
        const cxd xs = {__shfl(x.re, s), __shfl(x.im, s)};
        if (r < s) x -= D[r][s] * xs;
      }
      if (r < nb) Uinv[r * LU_NB + c] = x;
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

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Row permutation of the factorisation: the interchanges ipiv[0..n) applied in order to the
// identity, perm[i] = the row of A that ends in row i. The swaps are a sequential chain, so one
// thread applies them in LDS (n <= LU_PERM_LDS) and the workgroup writes the result out.
__global__ __launch_bounds__(256) void k_lu_perm(const int* __restrict__ ipiv, int n, int* __restrict__ perm) {
  __shared__ int q[LU_PERM_LDS];
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < n; ++j) {
      const int p = ipiv[j];
      const int t = q[j];
      q[j] = q[p];
      q[p] = t;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = q[i];
}

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

// U rows [r0, r0 + nb) over columns [c0, c0 + w): A[r0.., c0..] = L^-1 A[r0.., c0..], L^-1 the inverted
// unit-lower diagonal block Li (the block is copied out first: the GEMM writes where it reads)
static void lu_urows(hipStream_t st, cxd* A, int64_t lda, int r0, int nb, int c0, int w, const cxd* Li, cxd* work) {
  if (w <= 0) return;
  hipLaunchKernelGGL(k_copy2d, dim3(nblocks((int64_t)nb * w, 256)), dim3(256), 0, st, A + (int64_t)r0 * lda + c0, lda,
                     work, (int64_t)w, nb, w);
  gemm_rm(st, nb, w, nb, Li, LU_NB, work, w, A + (int64_t)r0 * lda + c0, lda, 0, 0);
}

constexpr int LU_GROUP = 4;

void lu_factor(hipStream_t st, DenseLU& F, cxd* work, bool device_perm) {
  const int n = F.n;
  const int64_t lda = F.lda;
  cxd* A = F.A;
  if (device_perm && n > LU_PERM_LDS) throw Error(VSIE_E_ARG, "dense LU: device permutation limited to n <= 8192");
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, F.d_info, 1, 0);
  // one panel of nb columns at k: pivots and rank-one updates inside it, its interchanges applied
  // to every other column, inverses of its diagonal triangles
  auto panel = [&](int k, int nb) {
    const int kend = k + nb;
    // pivot candidates of the next column live in the front of work (free until the U rows)
    double* pv = reinterpret_cast<double*>(work);
    int* pi = reinterpret_cast<int*>(pv + (n + 3) / 4);
    for (int j = k; j < kend; ++j) {
      if (j == k)
        hipLaunchKernelGGL(k_lu_pivot, dim3(1), dim3(1024), 0, st, A, lda, n, j, k, kend, F.d_ipiv, F.d_info);
      else
        hipLaunchKernelGGL(k_lu_pivot_parts, dim3(1), dim3(1024), 0, st, A, lda, n, j, k, kend, pv, pi,
                           (int)nblocks(n - j, 4), F.d_ipiv, F.d_info);
      if (j + 1 < n)
        hipLaunchKernelGGL(k_lu_rank1, dim3(nblocks(n - j - 1, 4)), dim3(256), 0, st, A, lda, n, j, kend,
                           j + 1 < kend ? pv : nullptr, pi);
    }
    if (n > nb) hipLaunchKernelGGL(k_lu_laswp, dim3(nblocks(n - nb, 256)), dim3(256), 0, st, A, lda, n, k, kend, F.d_ipiv);
    const int64_t blk = (int64_t)(k / LU_NB) * LU_NB * LU_NB;
    hipLaunchKernelGGL(k_lu_tri_inv, dim3(1), dim3(1024), 0, st, A, lda, k, nb, F.Linv + blk, F.Uinv + blk);
  };
  // U rows of the group's panels [k, kq) over the columns [c0, c0 + w), panel by panel: each takes
  // the earlier panels' U rows in one GEMM, then its own L^-1
  auto group_urows = [&](int k, int kq, int c0, int w) {
    for (int kt = k; kt < kq; kt += LU_NB) {
      const int nbt = std::min(LU_NB, kq - kt);
      gemm_rm(st, nbt, w, kt - k, A + (int64_t)kt * lda + k, lda, A + (int64_t)k * lda + c0, lda,
              A + (int64_t)kt * lda + c0, lda, 1, 1);
      lu_urows(st, A, lda, kt, nbt, c0, w, F.Linv + (int64_t)(kt / LU_NB) * LU_NB * LU_NB, work);
    }
  };
  // LU_GROUP panels per step: each panel of the group is first brought up to date by the group's
  // earlier panels alone (left-looking inside the group), and the trailing matrix takes the whole
  // group in one update of depth kend - k, so A22 is read and written once per group instead of
  // once per panel. Row interchanges of later panels reach the columns of earlier ones and of the
  // trailing matrix through k_lu_laswp; the deferred updates are row-wise, so the result is that
  // of one-panel-at-a-time elimination.
  for (int k = 0; k < n; k += LU_GROUP * LU_NB) {
    const int kend = std::min(k + LU_GROUP * LU_NB, n);
    for (int kq = k; kq < kend; kq += LU_NB) {
      const int nbq = std::min(LU_NB, kend - kq);
      if (kq > k) {
        group_urows(k, kq, kq, nbq);
        gemm_rm(st, n - kq, nbq, kq - k, A + (int64_t)kq * lda + k, lda, A + (int64_t)k * lda + kq, lda,
                A + (int64_t)kq * lda + kq, lda, 1, 1);
      }
      panel(kq, nbq);
    }
    const int nr = n - kend;
    if (nr > 0) {
      group_urows(k, kend, kend, nr);
      gemm_rm(st, nr, nr, kend - k, A + (int64_t)kend * lda + k, lda, A + (int64_t)k * lda + kend, lda,
              A + (int64_t)kend * lda + kend, lda, 1, 1);
    }
  }
  VSIE_HIP(hipGetLastError());
  int info = 0;
  if (device_perm) {
    // nothing held on the host: the permutation is formed on the device, only info comes back
    if (n > 0) hipLaunchKernelGGL(k_lu_perm, dim3(1), dim3(256), 0, st, F.d_ipiv, n, F.d_perm);
    VSIE_HIP(hipGetLastError());
    VSIE_HIP(hipMemcpyAsync(&info, F.d_info, sizeof(int), hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipStreamSynchronize(st));
    if (info != 0)
      throw Error(VSIE_E_SINGULAR, "dense LU: exactly singular pivot in column " + std::to_string(info - 1));
    return;
  }
  std::vector<int> ipiv(n);
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
