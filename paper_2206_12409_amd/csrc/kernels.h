// Host-side launchers of the device kernels (kernels.hip).
#pragma once
#include <vector>
#include "vsie_internal.h"

namespace vsie {

struct GridDims {
  int n1, n2, n3;        // body grid
  int ne1, ne2, ne3;     // extended grid
  int ob1, ob2, ob3;     // body offset inside the extended grid
  int64_t nv, Ne;
};

// Tissue voxels of the body grid: one byte per voxel (1 = tissue) and, per x row r = i2 + n2 i3,
// the run [lo, hi) of i1 outside which the row holds no tissue (lo = hi = 0 for a row of air). A
// row with air inside its run stores ~lo (negative) in place of lo, and its bytes decide inside the
// run. Kernels that read x_b only where it couples load nothing outside the runs.
struct BodyMask {
  const uint8_t* vox;
  const int2* runs;   // [n3 n2]
};

// setup
void launch_generator(hipStream_t st, const GaussTab* gt, const int ne[3], double kappa, const CellRule& cr, cxd* oct);
void launch_embed_circulant(hipStream_t st, const cxd* oct, const int ne[3], const int P[3], cxd* full);
template <typename R> void launch_extract_octant(hipStream_t st, const cxd* full, const int P[3], double scale, cx<R>* spec);
void launch_zcc_dense(hipStream_t st, const RwgDev& A, const RwgDev& B, double k, int64_t row0, int64_t nrows, cxd* out);
constexpr int SYM_TB = 128;
void launch_zcc_packed(hipStream_t st, const RwgDev& A, double k, const int* tiles, int64_t tile0, int64_t ntiles,
                       cxd* out);
void launch_zcc_pairs(hipStream_t st, const RwgDev& A, const RwgDev& B, const int* pi, const int* pj, int64_t np,
                      double k, cxd* out);
void launch_pfft_wtw(hipStream_t st, const double* W, const int* base, const cxd* oct, const int ne[3], const int* pm,
                     const int* pn, int64_t np, cxd* out);
void launch_pfft_tw_voxels(hipStream_t st, const double* W, const int* base, const cxd* oct, const int ne[3],
                           const int* vox, const int* pn, int64_t np, cxd* out);
void launch_zbc_near(hipStream_t st, const RwgDev& B, const double* centres, const int* pn, int64_t np, double h,
                     double k, cxd* out);

// FFT
template <typename R>
void fft_rows(hipStream_t st, int L, bool fwd, const cx<R>* in, cx<R>* out, int n_in, int n_out, int64_t in_row,
              int64_t out_row, int64_t nrows, const cx<R>* tw);
template <typename R>
void fft_strided(hipStream_t st, int L, bool fwd, const cx<R>* in, cx<R>* out, int n_in, int n_out, int64_t in_stride,
                 int64_t out_stride, int n_lo, int64_t n_hi, int64_t in_hi, int64_t out_hi, const cx<R>* tw);
// fused z pass; lengths 64..1024 run candidate `cand` (0..2) of the z-pass tunings with its block
// order (pairs k2, k1 tile from zconv_order for the same candidate)
template <typename R>
void fft_z_conv(hipStream_t st, int L, cx<R>* buf, int n3, int P1, int P2, const cx<R>* spec, const cx<R>* tw,
                const int* order, int cand);
std::vector<int> zconv_order(int L, int P1, int P2, bool fp64, int cand);
bool zconv_candidate(int L, bool fp64, int cand);                 // candidate exists for this length
void zconv_shape(int L, bool fp64, int cand, int* v, int* np);   // its values per thread, pencils per block

// matvec
// the first forward pass along x with the grid sources (masked x_b and the pFFT projection of x_n,
// eq. (13), gathered per projection row into projv [nprojrows][3] first) formed on the fly: out
// rows [3][ne3][ne2][L]
template <typename R>
void fft_rows_grid(hipStream_t st, int L, const cx<R>* xb, const cx<R>* xn, BodyMask mask, const int* vox2row,
                   const uint8_t* rowhas, const int* rowptr, const int* rowrwg, const R* roww, int nprojrows,
                   cx<R>* projv, const GridDims& g, cx<R>* out, const cx<R>* tw);
template <typename R> void launch_body_out(hipStream_t st, const cx<R>* xb, const cx<R>* E, const cx<R>* dvchi,
                                           const uint8_t* mask, cx<R>* yb, const GridDims& g);
template <typename R> void launch_pfft_gather(hipStream_t st, const R* W, const int* base, const cx<R>* E, cx<R>* yn,
                                              int mn, const GridDims& g);
template <typename R> void launch_csr_add(hipStream_t st, const int* rowid, const int* rowptr, const int* col,
                                          const cx<R>* val, const cx<R>* x, cx<R>* y, int nrows);
// low-rank factors stored rank-major (A[l][i], K <= 256 ranks of length M)
template <typename R> void launch_lr_t(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* x, int64_t M, int K,
                                       cx<R>* part, int max_chunks, cx<R>* out);
template <typename R> void launch_lr_n_add(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* t, int64_t M,
                                           int K, cx<R>* y);
// one pass over V (K x M): out = V^H x and y += conj(V)^T s; part holds lr_dual_part_elems(M)
template <typename R> void launch_lr_dual(hipStream_t st, const cx<R>* V, int K, int64_t M, const cx<R>* x,
                                          const cx<R>* s, cx<R>* y, cx<R>* part, cx<R>* out);
int64_t lr_dual_part_elems(int64_t M);
template <typename R> void launch_gemv_rows(hipStream_t st, const cx<R>* A, const cx<R>* x, int64_t nrow, int64_t ncol,
                                            cx<R>* out, int accumulate);
// Batched strided complex GEMM, C(i,j) = sum_k A(i,k) B(k,j), with element (i,j) of batch b at
// X[i sr + j sc + b sb]. Up to three independent problems share one launch (blockIdx.z runs over
// their batches in turn). Optional mask on B (mask index = B's element index relative to the
// batch) and masked accumulation into C. Split-K use: batch b covers K indices [b K, b K + K)
// of a contraction of length ktot, the last batch taking the remainder.
template <typename R> struct GemmArgs {
  const cx<R>* A;
  int64_t sar, sac, sab;
  const cx<R>* B;
  int64_t sbr, sbc, sbb;
  cx<R>* C;
  int64_t scr, scc, scb;
  int M, N, K;
  int64_t ktot;           // > 0: split-K over batches
  const uint8_t* maskB;
  const uint8_t* maskC;   // non-null: C += maskC * AB (mask index = C's element index)
  int accumulate;
  int negate;             // store -AB (with accumulate: C -= AB)
};
template <typename R> struct GemmSet {
  GemmArgs<R> g[3];
  int nbatch[3];
  int nprob;
};

template <typename R> void launch_zgemm(hipStream_t st, const GemmSet<R>& S);

constexpr int TT_RMAX = 128;
constexpr int TT_KBATCH = 64;   // most split-K batches of the transpose contraction over (j1, i2)
template <typename R> struct TTDesc {
  const cx<R>* G1[3];   // [n1][r1]
  const cx<R>* G2[3];   // [r1][n2][r2]
  const cx<R>* G3[3];   // [r2][n3][r3]
  const cx<R>* G4[3];   // [r3][m_f]
  int r1[3], r2[3], r3[3];
};
// forward and transpose far coupling of all three components, y_b += mask Zt x_f and
// y_f += sum_c Zt_c^T (mask x_b): launch_tt_pre reads x, adds the transpose into y_f (which must
// already hold the rest of its product) and leaves the forward intermediates in the work buffer;
// launch_tt_post adds the forward part into y_b
template <typename R> void launch_tt_pre(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf, const cx<R>* xf,
                                         const cx<R>* xb, BodyMask mask, cx<R>* yf, cx<R>* work);
template <typename R> void launch_tt_post(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                          const uint8_t* mask, cx<R>* yb, cx<R>* work);
// the halves used by the reduced (far-eliminated) operator: the transpose chain alone (s3 at the
// start of the work buffer), the forward chain from given rank vectors u3[c][TT_RMAX] instead of
// G4 x_f, and the forward accumulation into y_b alone
template <typename R> void launch_tt_transpose_pre(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                   const cx<R>* xb, BodyMask mask, cx<R>* work);
template <typename R> void launch_tt_forward_from(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                  const cx<R>* u3, cx<R>* work);
template <typename R> void launch_tt_forward_post(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                  const uint8_t* mask, cx<R>* yb, cx<R>* work);
int64_t tt_work_elems(const int n[3], int mf);
// y = Z x for the symmetric far block stored as upper-triangle tiles (part: 2 SYM_TB per tile)
template <typename R> void launch_symv_tiles(hipStream_t st, const cx<R>* Zp, const int* tiles, int T, const cx<R>* x,
                                             int m, cx<R>* part);
template <typename R> void launch_symv_reduce(hipStream_t st, const cx<R>* part, int T, int m, cx<R>* y);
// the tile pass for nrhs (1..16) right-hand sides at once: column b of x at x + b ldx, its partials
// at part + b ldp (ldp >= 2 SYM_TB per tile); reduce each with launch_symv_reduce
template <typename R> void launch_symv_multi(hipStream_t st, const cx<R>* Zp, const int* tiles, int T, const cx<R>* x,
                                             int64_t ldx, int m, int nrhs, cx<R>* part, int64_t ldp);
template <typename R> void launch_scatter_rhs(hipStream_t st, const int* idx, const double* vre, const double* vim,
                                             int ne, cx<R>* b);

// elimination of the far currents (FP64)
void launch_set_identity(hipStream_t st, cxd* X, int n);
void launch_unpack_sym(hipStream_t st, const cxd* Zp, int T, int m, cxd* out);
void launch_pack_sym(hipStream_t st, const cxd* X, int m, const int* tiles, int64_t ntiles, cxd* Zp);
void launch_build_far_factors(hipStream_t st, const cxd* V, int ka, const TTDesc<double>& T, int mf, int K, cxd* L);
template <typename R>
void launch_schur_apply(hipStream_t st, const cx<R>* S, int K, int ka, const int r3[3], const cx<R>* ta,
                        const cx<R>* s3, R sign, cx<R>* pa, cx<R>* p3);
void launch_schur_gather(hipStream_t st, int K, int ka, const int r3[3], const cxd* ta, const cxd* s3, double sign,
                         cxd* out);
void launch_schur_scatter(hipStream_t st, int K, int ka, const int r3[3], const cxd* in, double sign, cxd* pa,
                          cxd* p3);
template <typename R> void launch_mul_diag(hipStream_t st, const cx<R>* x, const cx<R>* d, cx<R>* y, int64_t n);
void launch_gather_idx(hipStream_t st, const cxd* src, const int* idx, int64_t n, cxd* dst);
void launch_scatter_idx(hipStream_t st, const cxd* src, const int* idx, int64_t n, cxd* dst);

// solver
// part[blk][nvec (+3)]: partial V^H w, and with_norm the partial |w|^2 of [0, s1), [s1, s2), [s2, n)
void launch_multidot(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* w, int64_t n, int64_t s1,
                     int64_t s2, int with_norm, cxd* part, int nblk);
void launch_sum_partials(hipStream_t st, const cxd* part, int nblk, int K, cxd* out);
// w -= V h (h on the device, nvec <= 1024) with part[blk][3] = partial |w|^2 of the three segments
void launch_multiaxpy_norm(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* h, cxd* w, int64_t n,
                          int64_t s1, int64_t s2, cxd* part, int nblk);
void launch_combine_add(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* y, cxd* x, int64_t n);
void launch_scale_copy(hipStream_t st, const cxd* a, double s, cxd* b, int64_t n);
void launch_sub(hipStream_t st, const cxd* a, const cxd* b, cxd* c, int64_t n);
void launch_add(hipStream_t st, cxd* a, const cxd* b, int64_t n);
void launch_d2f(hipStream_t st, const cxd* a, cxf* b, int64_t n);
void launch_f2d(hipStream_t st, const cxf* a, cxd* b, int64_t n);
void launch_norm_partial(hipStream_t st, const cxd* a, int64_t n, int64_t s1, int64_t s2, double* part, int nblk);

}  // namespace vsie
