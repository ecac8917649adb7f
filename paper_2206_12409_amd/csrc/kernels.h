// Host-side launchers of the device kernels (kernels.hip).
#pragma once
#include "vsie_internal.h"

namespace vsie {

struct GridDims {
  int n1, n2, n3;        // body grid
  int ne1, ne2, ne3;     // extended grid
  int ob1, ob2, ob3;     // body offset inside the extended grid
  int64_t nv, Ne;
};

// setup
void launch_generator(hipStream_t st, const GaussTab* gt, const int ne[3], double kappa, const CellRule& cr, cxd* oct);
void launch_embed_circulant(hipStream_t st, const cxd* oct, const int ne[3], const int P[3], cxd* full);
template <typename R> void launch_extract_octant(hipStream_t st, const cxd* full, const int P[3], double scale, cx<R>* spec);
void launch_zcc_dense(hipStream_t st, const RwgDev& A, const RwgDev& B, double k, int64_t row0, int64_t nrows, cxd* out);
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
template <typename R>
void fft_z_conv(hipStream_t st, int L, cx<R>* buf, int n3, int P1, int P2, const cx<R>* spec, const cx<R>* tw);

// matvec
template <typename R> void launch_build_grid(hipStream_t st, const cx<R>* xb, const cx<R>* xn, const uint8_t* mask,
                                             const int* vox2row, const int* rowptr, const int* rowrwg, const R* roww,
                                             cx<R>* grid, const GridDims& g);
template <typename R> void launch_body_out(hipStream_t st, const cx<R>* xb, const cx<R>* E, const cx<R>* dvchi,
                                           const uint8_t* mask, cx<R>* yb, const GridDims& g);
template <typename R> void launch_pfft_gather(hipStream_t st, const R* W, const int* base, const cx<R>* E, cx<R>* yn,
                                              int mn, const GridDims& g);
template <typename R> void launch_csr_add(hipStream_t st, const int* rowid, const int* rowptr, const int* col,
                                          const cx<R>* val, const cx<R>* x, cx<R>* y, int nrows);
template <typename R> void launch_tall_t(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* x, int64_t M, int K,
                                         cx<R>* part, int nblk, cx<R>* out);
template <typename R> void launch_tall_n_add(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* t, int64_t M,
                                             int K, cx<R>* y);
template <typename R> void launch_gemv_rows(hipStream_t st, const cx<R>* A, const cx<R>* x, int64_t nrow, int64_t ncol,
                                            cx<R>* out, int accumulate);
template <typename R> void launch_tt_forward(hipStream_t st, cx<R>* const G[4], const int r[3], const int n[3], int mf,
                                             const cx<R>* xf, const uint8_t* mask, cx<R>* yb, cx<R>* work);
template <typename R> void launch_tt_transpose(hipStream_t st, cx<R>* const G[4], const int r[3], const int n[3], int mf,
                                               const cx<R>* xb, const uint8_t* mask, cx<R>* yf, cx<R>* work);
template <typename R> void launch_scatter_rhs(hipStream_t st, const int* idx, const double* vre, const double* vim,
                                             int ne, cx<R>* b);

// solver
void launch_multidot(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* w, int64_t n, cxd* part, int nblk);
void launch_multiaxpy(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* h, cxd* w, int64_t n);
void launch_combine_add(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* y, cxd* x, int64_t n);
void launch_scale_copy(hipStream_t st, const cxd* a, double s, cxd* b, int64_t n);
void launch_sub(hipStream_t st, const cxd* a, const cxd* b, cxd* c, int64_t n);
void launch_add(hipStream_t st, cxd* a, const cxd* b, int64_t n);
void launch_d2f(hipStream_t st, const cxd* a, cxf* b, int64_t n);
void launch_f2d(hipStream_t st, const cxf* a, cxd* b, int64_t n);
void launch_norm_partial(hipStream_t st, const cxd* a, int64_t n, int64_t s1, int64_t s2, double* part, int nblk);

}  // namespace vsie
