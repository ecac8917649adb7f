// Device kernels of the hybrid VSIE library (gfx950).
//
//   setup:   Toeplitz generator of the volume operator on the extended-grid octant, circulant
//            embedding, EFIE entries (dense block and pair lists), pFFT precorrection entries,
//            near-rule coupling entries;
//   FFT:     LDS-staged Stockham radix-4/2 passes (contiguous rows, strided pencils) and the fused
//            z pass: forward FFT -> 3x3 symmetric spectral multiply -> inverse FFT;
//   matvec:  grid build (body embed + pFFT projection), body epilogue, pFFT interpolation,
//            precorrection SpMV, ACA, TT forward/transpose contractions, dense GEMV;
//   solver:  multi-dot, multi-axpy, norms and conversions for GMRES.
#include "kernels.h"

namespace vsie {

// Loads of data read once per product (the far-block tiles): the non-temporal hint keeps them
// from displacing reused data (x, partial sums) in the caches.
template <typename R> __device__ inline cx<R> ld_stream(const cx<R>* p) {
  return cx<R>{__builtin_nontemporal_load(&p->re), __builtin_nontemporal_load(&p->im)};
}


// =============================================================================================
// Setup kernels
// =============================================================================================

__global__ void k_generator_octant(const GaussTab* __restrict__ gt, int ne1, int ne2, int ne3, double kappa,
                                   CellRule cr, cxd* __restrict__ oct) {
  const int64_t S = (int64_t)ne1 * ne2 * ne3;
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= S) return;
  int d1 = (int)(id % ne1);
  int d2 = (int)((id / ne1) % ne2);
  int d3 = (int)(id / ((int64_t)ne1 * ne2));
  cxd T[6];
  generator_T(*gt, d1, d2, d3, kappa, cr, T);
  for (int c = 0; c < 6; ++c) oct[c * S + id] = T[c];
}

// full circulant grid t_c(n) for n in [0,P)^3, from the octant with the component parities
__global__ void k_embed_circulant(const cxd* __restrict__ oct, int ne1, int ne2, int ne3, int P1, int P2, int P3,
                                  cxd* __restrict__ full) {
  const int64_t PT = (int64_t)P1 * P2 * P3;
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= PT) return;
  int n1 = (int)(id % P1), n2 = (int)((id / P1) % P2), n3 = (int)(id / ((int64_t)P1 * P2));
  auto off = [](int nn, int P, int ne, int* d) -> bool {
    if (nn < ne) { *d = nn; return true; }
    if (nn > P - ne) { *d = nn - P; return true; }
    return false;
  };
  int d1, d2, d3;
  bool ok = off(n1, P1, ne1, &d1) && off(n2, P2, ne2, &d2) && off(n3, P3, ne3, &d3);
  const int64_t S = (int64_t)ne1 * ne2 * ne3;
  for (int c = 0; c < 6; ++c) {
    cxd v = {0.0, 0.0};
    if (ok) {
      int a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2, a3 = d3 < 0 ? -d3 : d3;
      v = oct[c * S + a1 + (int64_t)ne1 * (a2 + (int64_t)ne2 * a3)];
      double s = 1.0;
      if (c == 3) s = (double)((d1 > 0) - (d1 < 0)) * ((d2 > 0) - (d2 < 0));
      if (c == 4) s = (double)((d1 > 0) - (d1 < 0)) * ((d3 > 0) - (d3 < 0));
      if (c == 5) s = (double)((d2 > 0) - (d2 < 0)) * ((d3 > 0) - (d3 < 0));
      v = s * v;
    }
    full[c * PT + id] = v;
  }
}

template <typename R>
__global__ void k_extract_octant(const cxd* __restrict__ full, int P1, int P2, int P3, double scale,
                                 cx<R>* __restrict__ spec) {
  const int S1 = P1 / 2 + 1, S2 = P2 / 2 + 1, S3 = P3 / 2 + 1;
  const int64_t SO = (int64_t)S1 * S2 * S3;
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= SO) return;
  // output layout [f2][f1][6][f3]: for a z pencil (fixed f1, f2) each of the six components is a
  // contiguous run over f3, so the lanes of a wavefront (consecutive frequencies) read whole cache
  // lines
  const int f3 = (int)(id % S3);
  const int64_t pen = id / S3;
  const int f1 = (int)(pen % S1), f2 = (int)(pen / S1);
  const int64_t PT = (int64_t)P1 * P2 * P3;
  int64_t src = f1 + (int64_t)P1 * (f2 + (int64_t)P2 * f3);
  for (int c = 0; c < 6; ++c) {
    cxd v = full[c * PT + src];
    spec[(pen * 6 + c) * S3 + f3] = cx<R>{(R)(v.re * scale), (R)(v.im * scale)};
  }
}

// EFIE entry of two RWG functions (testing m of A, source n of B): sum over the four triangle
// pairs of s_a s_b [ -k^2 l_m l_n / (4 A_a A_b) Am[fa][fb] + l_m l_n / (A_a A_b) Bm ]
__device__ __host__ inline cxd rwg_pair_entry(const RwgDev& A, int m, const RwgDev& B, int n, double k) {
  cxd acc = {0, 0};
  for (int sa = 0; sa < 2; ++sa) {
    int ta = A.tpm[2 * m + sa];
    int fa = A.flpm[2 * m + sa];
    V3 va[3];
    for (int q = 0; q < 3; ++q) {
      int v = A.tris[3 * ta + q];
      va[q] = {A.verts[3 * v], A.verts[3 * v + 1], A.verts[3 * v + 2]};
    }
    double Aa = A.area[ta];
    for (int sb = 0; sb < 2; ++sb) {
      int tb = B.tpm[2 * n + sb];
      int fb = B.flpm[2 * n + sb];
      V3 vb[3];
      for (int q = 0; q < 3; ++q) {
        int v = B.tris[3 * tb + q];
        vb[q] = {B.verts[3 * v], B.verts[3 * v + 1], B.verts[3 * v + 2]};
      }
      double Ab = B.area[tb];
      cxd Bm, Am[3][3];
      tri_pair_moments(va, vb, Aa, Ab, k, &Bm, Am);
      double sg = (sa == sb) ? 1.0 : -1.0;
      double ll = A.len[m] * B.len[n];
      cxd term = (-(k * k) * ll / (4.0 * Aa * Ab)) * Am[fa][fb];
      term += (ll / (Aa * Ab)) * Bm;
      acc += sg * term;
    }
  }
  return acc;
}

__global__ void k_zcc_dense(RwgDev A, RwgDev B, double k, int64_t row0, int64_t nrows, cxd* __restrict__ out) {
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nrows * B.m) return;
  int m = (int)(row0 + id / B.m);
  int n = (int)(id % B.m);
  out[id] = rwg_pair_entry(A, m, B, n, k);
}

// upper-triangle tiles (I <= J) of the symmetric far block, each tile row-major SYM_TB x SYM_TB,
// zero-padded beyond m; diagonal tiles are stored in full
__global__ void k_zcc_packed(RwgDev A, double k, const int* __restrict__ tiles, int64_t tile0, int64_t ntiles,
                             cxd* __restrict__ out) {
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)SYM_TB * SYM_TB;
  if (id >= ntiles * per) return;
  const int64_t t = tile0 + id / per;
  const int e = (int)(id % per);
  const int m = tiles[2 * t] * SYM_TB + e / SYM_TB;
  const int n = tiles[2 * t + 1] * SYM_TB + e % SYM_TB;
  cxd v = {0, 0};
  if (m < A.m && n < A.m) v = rwg_pair_entry(A, m, A, n, k);
  out[id] = v;
}

__global__ void k_zcc_pairs(RwgDev A, RwgDev B, const int* __restrict__ pi, const int* __restrict__ pj, int64_t np,
                            double k, cxd* __restrict__ out) {
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= np) return;
  out[id] = rwg_pair_entry(A, pi[id], B, pj[id], k);
}

__device__ inline void T_lookup(const cxd* __restrict__ oct, int ne1, int ne2, int ne3, int d1, int d2, int d3,
                                cxd T[6]) {
  const int64_t S = (int64_t)ne1 * ne2 * ne3;
  int a1 = d1 < 0 ? -d1 : d1, a2 = d2 < 0 ? -d2 : d2, a3 = d3 < 0 ? -d3 : d3;
  int64_t idx = a1 + (int64_t)ne1 * (a2 + (int64_t)ne2 * a3);
  double s1 = (double)((d1 > 0) - (d1 < 0)), s2 = (double)((d2 > 0) - (d2 < 0)), s3 = (double)((d3 > 0) - (d3 < 0));
  T[0] = oct[idx];
  T[1] = oct[S + idx];
  T[2] = oct[2 * S + idx];
  T[3] = (s1 * s2) * oct[3 * S + idx];
  T[4] = (s1 * s3) * oct[4 * S + idx];
  T[5] = (s2 * s3) * oct[5 * S + idx];
}

__device__ inline void T_apply(const cxd T[6], const double w[3], cxd out[3]) {
  out[0] = w[0] * T[0] + w[1] * T[3] + w[2] * T[4];
  out[1] = w[0] * T[3] + w[1] * T[1] + w[2] * T[5];
  out[2] = w[0] * T[4] + w[1] * T[5] + w[2] * T[2];
}

// Grid interaction of two near RWG functions, sum_u sum_v W_m(u) . T(u - v) W_n(v) (dimensionless
// generator; the caller scales by h^3). One block per pair.
__global__ __launch_bounds__(256) void k_pfft_wtw_pairs(const double* __restrict__ W, const int* __restrict__ base,
                                                        const cxd* __restrict__ oct, int ne1, int ne2, int ne3,
                                                        const int* __restrict__ pm, const int* __restrict__ pn,
                                                        cxd* __restrict__ out) {
  __shared__ double wm[375], wn[375];
  __shared__ double red[2][256];
  const int pair = blockIdx.x;
  const int m = pm[pair], n = pn[pair];
  for (int e = threadIdx.x; e < 375; e += 256) {
    wm[e] = W[(int64_t)m * 375 + e];
    wn[e] = W[(int64_t)n * 375 + e];
  }
  __syncthreads();
  const int bm1 = base[3 * m], bm2 = base[3 * m + 1], bm3 = base[3 * m + 2];
  const int bn1 = base[3 * n], bn2 = base[3 * n + 1], bn3 = base[3 * n + 2];
  cxd acc = {0, 0};
  const int t = threadIdx.x;
  if (t < 250) {
    int u = t % 125, half = t / 125;
    int u1 = u % 5, u2 = (u / 5) % 5, u3 = u / 25;
    double w_u[3] = {wm[u], wm[125 + u], wm[250 + u]};
    cxd f[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int v = half; v < 125; v += 2) {
      int v1 = v % 5, v2 = (v / 5) % 5, v3 = v / 25;
      cxd T[6];
      T_lookup(oct, ne1, ne2, ne3, (bm1 + u1) - (bn1 + v1), (bm2 + u2) - (bn2 + v2), (bm3 + u3) - (bn3 + v3), T);
      double w_v[3] = {wn[v], wn[125 + v], wn[250 + v]};
      cxd o[3];
      T_apply(T, w_v, o);
      f[0] += o[0];
      f[1] += o[1];
      f[2] += o[2];
    }
    acc = w_u[0] * f[0] + w_u[1] * f[1] + w_u[2] * f[2];
  }
  red[0][t] = acc.re;
  red[1][t] = acc.im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] += red[0][t + s];
      red[1][t] += red[1][t + s];
    }
    __syncthreads();
  }
  if (t == 0) out[pair] = cxd{red[0][0], red[1][0]};
}

// Grid field of RWG n at voxel u (extended-grid coordinates): sum_v T(u - v) W_n(v) (dimensionless)
__global__ void k_pfft_tw_voxels(const double* __restrict__ W, const int* __restrict__ base,
                                 const cxd* __restrict__ oct, int ne1, int ne2, int ne3,
                                 const int* __restrict__ vox /*[np][3] ext coords*/, const int* __restrict__ pn,
                                 int64_t np, cxd* __restrict__ out /*[np][3]*/) {
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= np) return;
  const int n = pn[id];
  const int u1 = vox[3 * id], u2 = vox[3 * id + 1], u3 = vox[3 * id + 2];
  const int b1 = base[3 * n], b2 = base[3 * n + 1], b3 = base[3 * n + 2];
  cxd f[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int v = 0; v < 125; ++v) {
    int v1 = v % 5, v2 = (v / 5) % 5, v3 = v / 25;
    cxd T[6];
    T_lookup(oct, ne1, ne2, ne3, u1 - (b1 + v1), u2 - (b2 + v2), u3 - (b3 + v3), T);
    double w_v[3] = {W[(int64_t)n * 375 + v], W[(int64_t)n * 375 + 125 + v], W[(int64_t)n * 375 + 250 + v]};
    cxd o[3];
    T_apply(T, w_v, o);
    f[0] += o[0];
    f[1] += o[1];
    f[2] += o[2];
  }
  out[3 * id] = f[0];
  out[3 * id + 1] = f[1];
  out[3 * id + 2] = f[2];
}

// Coupling entries with the near rule (8 volume x 5 surface points) for (voxel, RWG) pairs:
// Z_bc[p a, n] = - sum_i (h^3/8) sum_sides s (l/2) sum_q w_q [ D(r_i - r'_q) (r'_q - p_T) ]_a
__global__ void k_zbc_near_pairs(RwgDev B, const double* __restrict__ centres /*[np][3]*/, const int* __restrict__ pn,
                                 int64_t np, double h, double k, cxd* __restrict__ out /*[np][3]*/) {
  int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= np) return;
  const int n = pn[id];
  const double a = 0.5 / sqrt(3.0) * h;
  V3 c = {centres[3 * id], centres[3 * id + 1], centres[3 * id + 2]};
  cxd acc[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int side = 0; side < 2; ++side) {
    int t = B.tpm[2 * n + side];
    int fv = B.fpm[2 * n + side];
    double s = side == 0 ? 1.0 : -1.0;
    V3 tv[3];
    for (int q = 0; q < 3; ++q) {
      int v = B.tris[3 * t + q];
      tv[q] = {B.verts[3 * v], B.verts[3 * v + 1], B.verts[3 * v + 2]};
    }
    V3 pf = {B.verts[3 * fv], B.verts[3 * fv + 1], B.verts[3 * fv + 2]};
    for (int q = 0; q < 5; ++q) {
      double l[3], w;
      r5_point(q, l, &w);
      V3 rs = l[0] * tv[0] + l[1] * tv[1] + l[2] * tv[2];
      V3 fvv = (w * s * 0.5 * B.len[n]) * (rs - pf);
      cxd fv3[3] = {{fvv.x, 0}, {fvv.y, 0}, {fvv.z, 0}};
      for (int iz = 0; iz < 2; ++iz)
        for (int iy = 0; iy < 2; ++iy)
          for (int ix = 0; ix < 2; ++ix) {
            V3 r = {c.x + (ix ? a : -a), c.y + (iy ? a : -a), c.z + (iz ? a : -a)};
            cxd o[3];
            dyad_apply(r - rs, fv3, k, o);
            acc[0] += o[0];
            acc[1] += o[1];
            acc[2] += o[2];
          }
    }
  }
  const double wv = -h * h * h / 8.0;
  out[3 * id] = wv * acc[0];
  out[3 * id + 1] = wv * acc[1];
  out[3 * id + 2] = wv * acc[2];
}

// =============================================================================================
// FFT (Stockham autosort, radix 4 with a final radix-2 stage when log2 L is odd)
// =============================================================================================

template <typename R, int L, int NP, bool FWD>
__device__ inline void lds_fft(cx<R>* sm, const cx<R>* __restrict__ tw, int tid) {
  constexpr int LP = L + 1;
  constexpr int NB4 = (NP * (L / 4) + 255) / 256;
  constexpr int NB2 = (NP * (L / 2) + 255) / 256;
  int Ls = 1;
#pragma unroll 1
  for (; Ls * 4 <= L; Ls *= 4) {
    cx<R> v[NB4][4];
    const int tstep = L / (4 * Ls);
#pragma unroll
    for (int u = 0; u < NB4; ++u) {
      int b = tid + u * 256;
      if (b < NP * (L / 4)) {
        int p = b / (L / 4), j = b % (L / 4);
        int kk = j & (Ls - 1);
        cx<R>* s = sm + p * LP;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cx<R> a = s[j + q * (L / 4)];
          if (q) {
            cx<R> w = tw[(q * kk * tstep) & (L - 1)];
            if (!FWD) w.im = -w.im;
            a = a * w;
          }
          v[u][q] = a;
        }
        cx<R> t0 = v[u][0] + v[u][2], t1 = v[u][0] - v[u][2], t2 = v[u][1] + v[u][3], d = v[u][1] - v[u][3];
        cx<R> t3 = FWD ? cx<R>{d.im, -d.re} : cx<R>{-d.im, d.re};
        v[u][0] = t0 + t2;
        v[u][1] = t1 + t3;
        v[u][2] = t0 - t2;
        v[u][3] = t1 - t3;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB4; ++u) {
      int b = tid + u * 256;
      if (b < NP * (L / 4)) {
        int p = b / (L / 4), j = b % (L / 4);
        int kk = j & (Ls - 1);
        cx<R>* s = sm + p * LP;
        int base = (j - kk) * 4 + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) s[base + q * Ls] = v[u][q];
      }
    }
    __syncthreads();
  }
  if (Ls < L) {
    cx<R> v[NB2][2];
    const int tstep = L / (2 * Ls);
#pragma unroll
    for (int u = 0; u < NB2; ++u) {
      int b = tid + u * 256;
      if (b < NP * (L / 2)) {
        int p = b / (L / 2), j = b % (L / 2);
        int kk = j & (Ls - 1);
        cx<R>* s = sm + p * LP;
        cx<R> a0 = s[j], a1 = s[j + L / 2];
        cx<R> w = tw[(kk * tstep) & (L - 1)];
        if (!FWD) w.im = -w.im;
        a1 = a1 * w;
        v[u][0] = a0 + a1;
        v[u][1] = a0 - a1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB2; ++u) {
      int b = tid + u * 256;
      if (b < NP * (L / 2)) {
        int p = b / (L / 2), j = b % (L / 2);
        int kk = j & (Ls - 1);
        cx<R>* s = sm + p * LP;
        int base = (j - kk) * 2 + kk;
        s[base] = v[u][0];
        s[base + Ls] = v[u][1];
      }
    }
    __syncthreads();
  }
}

// Fused z pass on buf[3][n3][P2][P1]: forward FFT of length L = P3 over the n3 stored planes,
// y_a(k) = sum_b T_ab(k) x_b(k) with the octant-folded spectra, inverse FFT, first n3 outputs
// written back in place. TP adjacent pencils per block; one component at a time occupies LDS
// while the transformed components wait in registers (each thread owns the same (pencil, k3)
// slots in every component, so the 3x3 multiply is thread-local).
template <typename R, int L, int TP>
__global__ __launch_bounds__(256) void k_fft_z_conv(cx<R>* __restrict__ buf, int n3, int P1, int P2,
                                                    const cx<R>* __restrict__ spec, const cx<R>* __restrict__ tw) {
  constexpr int EPT = (TP * L + 255) / 256;
  __shared__ cx<R> sm[TP * (L + 1)];
  const int tid = threadIdx.x;
  const int tiles = (P1 + TP - 1) / TP;
  const int k2 = blockIdx.x / tiles;
  const int k1_0 = (blockIdx.x % tiles) * TP;
  const int64_t plane = (int64_t)P1 * P2;
  const int64_t comp = plane * n3;
  cx<R> X[3][EPT];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    for (int e = tid; e < TP * L; e += 256) {
      int p = e % TP, i = e / TP;
      cx<R> v = {0, 0};
      if (i < n3 && k1_0 + p < P1) v = buf[c * comp + (int64_t)i * plane + (int64_t)k2 * P1 + k1_0 + p];
      sm[p * (L + 1) + i] = v;
    }
    __syncthreads();
    lds_fft<R, L, TP, true>(sm, tw, tid);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      int e = tid + u * 256;
      if (e < TP * L) X[c][u] = sm[(e % TP) * (L + 1) + e / TP];
    }
    __syncthreads();
  }
  const int S1 = P1 / 2 + 1, S3 = L / 2 + 1;
  const int f2 = k2 <= P2 / 2 ? k2 : P2 - k2;
  const R s2 = k2 <= P2 / 2 ? (R)1 : (R)-1;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    int e = tid + u * 256;
    int p = e % TP, k3 = e / TP;
    int k1 = k1_0 + p;
    if (e >= TP * L || k1 >= P1) continue;
    int f1 = k1 <= P1 / 2 ? k1 : P1 - k1;
    int f3 = k3 <= L / 2 ? k3 : L - k3;
    R s1 = k1 <= P1 / 2 ? (R)1 : (R)-1;
    R s3 = k3 <= L / 2 ? (R)1 : (R)-1;
    const cx<R>* rec = spec + 6 * ((int64_t)f2 * S1 + f1) * S3 + f3;
    cx<R> Txx = rec[0], Tyy = rec[S3], Tzz = rec[2 * S3];
    cx<R> Txy = (s1 * s2) * rec[3 * S3];
    cx<R> Txz = (s1 * s3) * rec[4 * S3];
    cx<R> Tyz = (s2 * s3) * rec[5 * S3];
    cx<R> x = X[0][u], y = X[1][u], z = X[2][u];
    X[0][u] = Txx * x + Txy * y + Txz * z;
    X[1][u] = Txy * x + Tyy * y + Tyz * z;
    X[2][u] = Txz * x + Tyz * y + Tzz * z;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      int e = tid + u * 256;
      if (e < TP * L) sm[(e % TP) * (L + 1) + e / TP] = X[c][u];
    }
    __syncthreads();
    lds_fft<R, L, TP, false>(sm, tw, tid);
    for (int e = tid; e < TP * n3; e += 256) {
      int p = e % TP, i = e / TP;
      if (k1_0 + p < P1) buf[c * comp + (int64_t)i * plane + (int64_t)k2 * P1 + k1_0 + p] = sm[p * (L + 1) + i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// Two-level register FFT of length L = A * B (A >= B): thread j < B loads x[j + B m], m < A, and
// transforms over m in registers; after the twiddle w_L^(j k1) one LDS transpose hands thread
// k1 < A the values over j, which it transforms in registers to X[k1 + A k2]. Global loads and
// stores go straight from/to registers; the transpose is the only LDS traffic (its padding is
// chosen per lane layout to keep the banks apart).
__host__ __device__ constexpr int bitrev_of(int m, int n) {
  int r = 0;
  for (int b = 1, hi = n >> 1; b < n; b <<= 1, hi >>= 1)
    if (m & b) r |= hi;
  return r;
}

template <typename R, int N, int L, bool FWD>
__device__ inline void reg_dft(cx<R>* v, const cx<R>* __restrict__ tw) {
#pragma unroll
  for (int ln = 2; ln <= N; ln <<= 1) {
#pragma unroll
    for (int i = 0; i < N; i += ln) {
#pragma unroll
      for (int j = 0; j < ln / 2; ++j) {
        cx<R> t = v[i + j + ln / 2];
        if (j != 0) {
          cx<R> w = tw[(j * (N / ln)) * (L / N)];
          if (!FWD) w.im = -w.im;
          t = w * t;
        }
        cx<R> u = v[i + j];
        v[i + j] = u + t;
        v[i + j + ln / 2] = u - t;
      }
    }
  }
}

// Sources of the extended grid (eq. (13)): masked body currents plus the pFFT projection of the
// near currents, which a voxel-keyed CSR (one row of weights per grid voxel that any stencil
// touches) gathers into projv[row][3] first. Read in place of a stored grid by the first forward
// pass.
template <typename R> struct GridSrc {
  const cx<R>* xb;
  const uint8_t* mask;
  const int2* runs;        // tissue run of each body x row (BodyMask)
  const int* vox2row;
  const uint8_t* rowhas;   // per x row (i2 + ne2 i3): any projection voxel in it
  const cx<R>* projv;
  GridDims g;
};

// projv[r][c] = sum_e roww[e][c] x_n[rwg(e)] over CSR row r: four lanes per projection row, each
// summing every fourth entry, combined by two lane exchanges (fixed order)
template <typename R>
__global__ __launch_bounds__(256) void k_proj_rows(const int* __restrict__ rowptr, const int* __restrict__ rowrwg,
                                                   const R* __restrict__ roww, const cx<R>* __restrict__ xn,
                                                   int nrows, cx<R>* __restrict__ projv) {
  const int r = blockIdx.x * 64 + threadIdx.x / 4, sub = threadIdx.x % 4;
  const bool live = r < nrows;
  R a[6] = {0, 0, 0, 0, 0, 0};
  if (live)
    for (int e = rowptr[r] + sub; e < rowptr[r + 1]; e += 4) {
      const cx<R> j = xn[rowrwg[e]];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const R w = roww[3 * (int64_t)e + q];
        a[2 * q] += w * j.re;
        a[2 * q + 1] += w * j.im;
      }
    }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    a[q] += __shfl_xor(a[q], 1, 4);
    a[q] += __shfl_xor(a[q], 2, 4);
  }
  if (live && sub < 3) projv[3 * (int64_t)r + sub] = cx<R>{a[2 * sub], a[2 * sub + 1]};
}

// SRC: row-major forward pass over x whose input rows (c, i3, i2) are formed from the grid
// sources instead of read (the grid build fused into the first FFT pass).
template <typename R, int A, int B, int NP, bool FWD, bool STRIDED, bool SRC = false>
__global__ __launch_bounds__(NP * A) void k_fft2(const cx<R>* __restrict__ in, cx<R>* __restrict__ out, int n_in,
                                                 int n_out, int64_t in_stride, int64_t out_stride, int n_lo,
                                                 int64_t in_hi, int64_t out_hi, int64_t nrows,
                                                 const cx<R>* __restrict__ tw, GridSrc<R> gs) {
  static_assert(!SRC || (FWD && !STRIDED), "grid sources feed the forward row pass only");
  constexpr int L = A * B;
  // transpose rows of RS and pencils PS apart (16-byte slots). Row-major pencils (lanes along a
  // pencil) need only the row padding; the strided form's lanes run across pencils, so their
  // offset is skewed too, which keeps its transpose stores and loads off shared banks
  constexpr int RS = A + (STRIDED ? (NP >= 16 ? 0 : (NP == 8 ? 8 : 4)) : 1);
  constexpr int PS = B * RS + (STRIDED ? (NP >= 8 ? 1 : 3) : 0);
  __shared__ cx<R> S[(NP - 1) * PS + B * RS];
  __shared__ cx<R> twl[L];   // twiddles staged once per block
  const int t = threadIdx.x;
  for (int k = t; k < L; k += NP * A) twl[k] = tw[k];
  __syncthreads();
  int p, u;
  const cx<R>* ib;
  cx<R>* ob;
  bool valid;
  if (STRIDED) {
    p = t % NP;
    u = t / NP;
    const int tiles = (n_lo + NP - 1) / NP;
    const int64_t hi = blockIdx.x / tiles;
    const int lo = (int)(blockIdx.x % tiles) * NP + p;
    valid = lo < n_lo;
    ib = in + hi * in_hi + lo;
    ob = out + hi * out_hi + lo;
  } else {
    u = t % A;
    p = t / A;
    const int64_t row = (int64_t)blockIdx.x * NP + p;
    valid = row < nrows;
    ib = in + row * in_hi;
    ob = out + row * out_hi;
  }
  cx<R>* Sp = S + p * PS;
  if (u < B) {
    const int j = u;
    cx<R> v[A];
    if constexpr (SRC) {
      // row = (c ne3 + i3) ne2 + i2; body voxel (n - ob1, i2 - ob2, i3 - ob3) when inside
      const GridDims& g = gs.g;
      const int64_t row = (int64_t)blockIdx.x * NP + p;
      const int plane = g.ne3 * g.ne2;
      const int c = valid ? (int)(row / plane) : 0;
      const int rem = valid ? (int)(row - (int64_t)c * plane) : 0;
      const int i3 = rem / g.ne2, i2 = rem - (rem / g.ne2) * g.ne2;
      const int b2 = i2 - g.ob2, b3 = i3 - g.ob3;
      const bool rin = valid && gs.xb && b2 >= 0 && b2 < g.n2 && b3 >= 0 && b3 < g.n3;
      const int64_t pb = (int64_t)g.n1 * (b2 + (int64_t)g.n2 * b3) - g.ob1;
      const int64_t vrow = (int64_t)g.ne1 * (i2 + (int64_t)g.ne2 * i3);
      const bool rproj = valid && gs.vox2row && gs.rowhas[i2 + (int64_t)g.ne2 * i3];
      const cx<R>* xbc = gs.xb + (int64_t)c * g.nv;
      // x_b is loaded only inside the row's tissue run (bytes tested only in a run with air
      // inside); every load of the row is issued before any is tested; the projection rows (voxels
      // next to the near conductors only) are walked afterwards
      const int2 run = rin ? gs.runs[b2 + (int64_t)g.n2 * b3] : int2{0, 0};
      const bool holes = run.x < 0;
      const int lo = holes ? ~run.x : run.x, hi = run.y;
      int pr[A];
#pragma unroll
      for (int m = 0; m < A; ++m) {
        const int n = j + B * m;
        const int b1 = n - g.ob1;
        const bool inb = rin && n < n_in && b1 >= lo && b1 < hi && b1 >= 0 && b1 < g.n1;
        const cx<R> xv = inb ? xbc[pb + n] : cx<R>{0, 0};
        const uint8_t mk = (inb && holes) ? gs.mask[pb + n] : (uint8_t)inb;
        v[bitrev_of(m, A)] = mk ? xv : cx<R>{0, 0};
        pr[m] = (rproj && n < n_in) ? gs.vox2row[vrow + n] : -1;
      }
#pragma unroll
      for (int m = 0; m < A; ++m)
        if (pr[m] >= 0) v[bitrev_of(m, A)] += gs.projv[3 * (int64_t)pr[m] + c];
    } else {
#pragma unroll
      for (int m = 0; m < A; ++m) {
        const int n = j + B * m;
        v[bitrev_of(m, A)] = (valid && n < n_in) ? ib[(int64_t)n * in_stride] : cx<R>{0, 0};
      }
    }
    reg_dft<R, A, L, FWD>(v, twl);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cx<R> w = twl[(j * k1) & (L - 1)];
      if (!FWD) w.im = -w.im;
      Sp[j * RS + k1] = (k1 == 0) ? v[k1] : v[k1] * w;
    }
  }
  __syncthreads();
  if (u < A) {
    const int k1 = u;
    cx<R> v[B];
#pragma unroll
    for (int j = 0; j < B; ++j) v[bitrev_of(j, B)] = Sp[j * RS + k1];
    reg_dft<R, B, L, FWD>(v, twl);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const int k = k1 + A * k2;
      if (valid && k < n_out) ob[(int64_t)k * out_stride] = v[k2];
    }
  }
}

// Fused z pass as a mixed-radix Stockham FFT whose first and last stages run in registers:
// T = L / V threads per pencil, V values per thread, NP pencils per block. Radices V, V, ...,
// then the remainder; a radix-R stage with sub-length Ls takes butterfly b < L / R from positions
// b + (L / R) q and writes position (b - b mod Ls) R + b mod Ls + q Ls. The last forward stage
// leaves thread j holding X[b + (L / R) q] for its butterflies b = j + T i, which are exactly the
// inputs of the first inverse stage (same radix), so the 3 x 3 spectral multiply sits between
// them without an exchange. Between stages one LDS exchange per component.
template <int L, int V> struct ZRad {   // radix of stage s of the forward transform (product = L)
  static constexpr int lg(int x) { return x <= 1 ? 0 : 1 + lg(x / 2); }
  static constexpr int nst = (lg(L) + lg(V) - 1) / lg(V);
  static constexpr int rad(int s) {
    int r = 1;
    for (int i = 0; i < nst - 1; ++i) r *= V;
    return (s + 1 < nst) ? V : L / r;
  }
};

// exchange barrier: the whole block, or only the wavefront when each pencil lives in one
// wavefront (LDS accesses of one wavefront complete in order; the fence keeps the compiler from
// moving them across)
template <bool WAVE> __device__ inline void zsync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// The same Stockham transform for pencils held by one thread group, with its LDS traffic laid out
// for the banks. Exchange slot a of a pencil row is stored at a ^ ((a >> log2 V) & 15): with
// 16-byte elements the stores of the early stages (sub-length 1 and V, lanes V or V^2 slots
// apart) otherwise fall on a few banks, while the swizzle keeps every load and store of every
// stage conflict-free and the row in place. A stage's twiddles w_L^(q kk tstep), q < RAD, come
// from one table entry w = w_L^(kk tstep) per butterfly (per-stage tables in LDS, consecutive
// lanes on consecutive entries) and its powers w^q by multiplication; the twiddles inside the
// small DFTs are exact constants (multiples of an eighth turn, or of a sixteenth for radix 16).
template <int L, int V> struct ZTw {
  using Z = ZRad<L, V>;
  // sub-length of forward stage s and of inverse stage u (the inverse runs the stages backwards)
  static constexpr int ls_fwd(int s) {
    int r = 1;
    for (int i = 0; i < s; ++i) r *= Z::rad(i);
    return r;
  }
  static constexpr int ls_inv(int u) {
    int r = 1;
    for (int i = 0; i < u; ++i) r *= Z::rad(Z::nst - 1 - i);
    return r;
  }
  // table offsets: forward stages 1.., then inverse stages 1.. (stage 0 has no twiddles)
  static constexpr int off_fwd(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += ls_fwd(i);
    return o;
  }
  static constexpr int n_fwd() { return off_fwd(Z::nst); }
  static constexpr int off_inv(int u) {
    int o = n_fwd();
    for (int i = 1; i < u; ++i) o += ls_inv(i);
    return o;
  }
  static constexpr int size() { return off_inv(Z::nst); }
};

static_assert(ZTw<256, 4>::size() == 168 && ZTw<128, 4>::size() == 126 && ZTw<1024, 16>::size() == 340,
              "per-stage twiddle table sizes");

template <int L, int V> __device__ inline int zswz(int a) {
  constexpr int S = ZRad<V, 2>::lg(V);
  return a ^ ((a >> S) & 15);
}

// fill the per-stage twiddle tables (all threads of the block, stride nthr) from w_L^m = tw[m]
template <typename R, int L, int V>
__device__ inline void ztw_fill(cx<R>* tws, const cx<R>* __restrict__ tw, int t, int nthr) {
  using Z = ZRad<L, V>;
  using W = ZTw<L, V>;
  for (int e = t; e < W::size(); e += nthr) {
    int ls = 1, rad = 1, k = 0;
#pragma unroll
    for (int s = 1; s < Z::nst; ++s)
      if (e >= W::off_fwd(s) && e < W::off_fwd(s) + W::ls_fwd(s)) {
        ls = W::ls_fwd(s);
        rad = Z::rad(s);
        k = e - W::off_fwd(s);
      }
#pragma unroll
    for (int u = 1; u < Z::nst; ++u)
      if (e >= W::off_inv(u) && e < W::off_inv(u) + W::ls_inv(u)) {
        ls = W::ls_inv(u);
        rad = Z::rad(Z::nst - 1 - u);
        k = e - W::off_inv(u);
      }
    tws[e] = tw[(k * (L / (rad * ls))) & (L - 1)];
  }
}

// w_RAD^m (forward sign), exact for RAD <= 16: multiples of 2 pi / 16 from three constants
template <typename R> __device__ inline cx<R> unit16(int m16) {
  constexpr R C1 = (R)0.92387953251128675613L;   // cos(pi / 8)
  constexpr R S1 = (R)0.38268343236508977173L;   // sin(pi / 8)
  constexpr R H = (R)0.70710678118654752440L;    // sqrt(1 / 2)
  const int m = m16 & 15;
  // first quadrant values of cos for m = 0..4
  const R cq[5] = {(R)1, C1, H, S1, (R)0};
  const int q = m >> 2, r = m & 3;
  R c = cq[r], s = cq[4 - r];   // cos and sin of 2 pi r / 16
  // rotate by q quarter turns: angle 2 pi m / 16 = q pi / 2 + 2 pi r / 16
  R cr = c, sr = s;
  if (q == 1) { cr = -s; sr = c; }
  else if (q == 2) { cr = -c; sr = -s; }
  else if (q == 3) { cr = s; sr = -c; }
  return cx<R>{cr, -sr};
}

template <typename R, int RAD, bool FWD>
__device__ inline void small_dft_c(cx<R>* a) {
  cx<R> v[RAD];
#pragma unroll
  for (int q = 0; q < RAD; ++q) v[bitrev_of(q, RAD)] = a[q];
#pragma unroll
  for (int ln = 2; ln <= RAD; ln <<= 1) {
#pragma unroll
    for (int i = 0; i < RAD; i += ln) {
#pragma unroll
      for (int j = 0; j < ln / 2; ++j) {
        cx<R> t = v[i + j + ln / 2];
        const int m16 = j * (16 / ln);   // w_ln^j = w_16^(16 j / ln)
        if (m16 == 4) {
          t = FWD ? cx<R>{t.im, -t.re} : cx<R>{-t.im, t.re};   // times -i (forward) or i
        } else if (m16 != 0) {
          cx<R> w = unit16<R>(m16);
          if (!FWD) w.im = -w.im;
          t = w * t;
        }
        const cx<R> u = v[i + j];
        v[i + j] = u + t;
        v[i + j + ln / 2] = u - t;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RAD; ++q) a[q] = v[q];
}

template <typename R, int L, int V, int RAD, bool FWD>
__device__ inline void zstage_c(cx<R>* v, int j, int Ls, const cx<R>* tw1) {
  constexpr int T = L / V;
  constexpr int NB = V / RAD;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = j + T * i;
    const int kk = b & (Ls - 1);
    cx<R>* a = v + i * RAD;
    if (Ls > 1) {
      cx<R> w1 = tw1[kk];
      if (!FWD) w1.im = -w1.im;
      cx<R> wq = w1;
#pragma unroll
      for (int q = 1; q < RAD; ++q) {
        a[q] = a[q] * wq;
        if (q + 1 < RAD) wq = wq * w1;
      }
    }
    small_dft_c<R, RAD, FWD>(a);
  }
}
template <typename R, int L, int V, int RAD>
__device__ inline void zstore_c(cx<R>* Sp, const cx<R>* v, int j, int Ls) {
  constexpr int T = L / V;
  constexpr int NB = V / RAD;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = j + T * i;
    const int kk = b & (Ls - 1);
    const int base = (b - kk) * RAD + kk;
#pragma unroll
    for (int q = 0; q < RAD; ++q) Sp[zswz<L, V>(base + q * Ls)] = v[i * RAD + q];
  }
}
template <typename R, int L, int V, int RAD>
__device__ inline void zload_c(const cx<R>* Sp, cx<R>* v, int j) {
  constexpr int T = L / V;
  constexpr int NB = V / RAD;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < RAD; ++q) v[i * RAD + q] = Sp[zswz<L, V>(j + T * i + (L / RAD) * q)];
}
template <typename R, int L, int V, bool FWD, int RAD>
__device__ inline void zstep_c(cx<R>* Sp, cx<R>* v, int j, int Ls, bool load, bool store, const cx<R>* tw1) {
  if (load) {
    zsync<true>();
    zload_c<R, L, V, RAD>(Sp, v, j);
  }
  zstage_c<R, L, V, RAD, FWD>(v, j, Ls, tw1);
  if (store) {
    if (load) zsync<true>();
    zstore_c<R, L, V, RAD>(Sp, v, j, Ls);
  }
}
template <typename R, int L, int V, bool FWD>
__device__ inline void zstep_any_c(int rad, cx<R>* Sp, cx<R>* v, int j, int Ls, bool load, bool store,
                                   const cx<R>* tw1) {
  if (rad == V) zstep_c<R, L, V, FWD, V>(Sp, v, j, Ls, load, store, tw1);
  else if (rad == V / 2 && V >= 4) zstep_c<R, L, V, FWD, (V >= 4 ? V / 2 : 2)>(Sp, v, j, Ls, load, store, tw1);
  else if (rad == V / 4 && V >= 8) zstep_c<R, L, V, FWD, (V >= 8 ? V / 4 : 2)>(Sp, v, j, Ls, load, store, tw1);
  else if (rad == V / 8 && V >= 16) zstep_c<R, L, V, FWD, (V >= 16 ? V / 8 : 2)>(Sp, v, j, Ls, load, store, tw1);
}
// the stage radices a length-L transform with V values per thread uses: V, then the remainder,
// which zstep_any_c covers down to V / 8
template <int L, int V> constexpr bool zradices_supported() {
  using Z = ZRad<L, V>;
  const int r = Z::rad(Z::nst - 1);
  return r == V || (r == V / 2 && V >= 4) || (r == V / 4 && V >= 8) || (r == V / 8 && V >= 16);
}
// all stages of one transform on a pencil row held by one wavefront (or part of one); tws: the
// per-stage twiddle tables (ZTw layout)
template <typename R, int L, int V, bool FWD>
__device__ inline void zfft_c(cx<R>* Sp, cx<R>* v, int j, const cx<R>* tws) {
  using Z = ZRad<L, V>;
  using W = ZTw<L, V>;
  int Ls = 1;
  if (FWD) {
#pragma unroll
    for (int s = 0; s < Z::nst; ++s) {
      zstep_any_c<R, L, V, true>(Z::rad(s), Sp, v, j, Ls, s > 0, s + 1 < Z::nst, tws + W::off_fwd(s));
      Ls *= Z::rad(s);
    }
  } else {
#pragma unroll
    for (int s = Z::nst - 1; s >= 0; --s) {
      const int u = Z::nst - 1 - s;
      zstep_any_c<R, L, V, false>(Z::rad(s), Sp, v, j, Ls, s < Z::nst - 1, s > 0, tws + W::off_inv(u));
      Ls *= Z::rad(s);
    }
  }
}

// Staging of a block's NP adjacent pencils between buf (pencil k1 at base + k1, plane n at
// + n plane, component c at + c comp) and the LDS rows S[p (L + 1) + n], one row per pencil that
// the three components take in turn. Thread t takes pencil t % NP and the planes
// t / NP + m NT / NP, with neighbouring threads on neighbouring pencils (coalesced). zstage_load
// issues the loads of all three components at once into registers, zstage_put stores one
// component into the rows, zstage_out writes one component's rows back. np_here: pencils of the
// block that exist.
template <int L, int NP, int NT> struct ZStage {
  static constexpr int NSTEP = NT / NP;
  static constexpr int MAXIT = (L / 2 + NSTEP - 1) / NSTEP;
};
template <typename R, int L, int NP, int NT, int M>
__device__ inline void zstage_load(cx<R> (&v)[3][M], const cx<R>* __restrict__ base, int t, int n3, int64_t plane,
                                   int64_t comp, int np_here) {
  using Z = ZStage<L, NP, NT>;
  static_assert(M == Z::MAXIT, "staging registers");
  const int p = t % NP, n0 = t / NP;
  const bool ok = p < np_here;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < Z::MAXIT; ++m) {
      const int n = n0 + m * Z::NSTEP;
      v[c][m] = (ok && n < n3) ? base[c * comp + (int64_t)n * plane + p] : cx<R>{0, 0};
    }
}
template <typename R, int L, int NP, int NT, int M>
__device__ inline void zstage_put(cx<R>* S, const cx<R> (&v)[M], int t, int n3) {
  using Z = ZStage<L, NP, NT>;
  static_assert(M == Z::MAXIT, "staging registers");
  const int p = t % NP, n0 = t / NP;
#pragma unroll
  for (int m = 0; m < Z::MAXIT; ++m) {
    const int n = n0 + m * Z::NSTEP;
    if (n < n3) S[p * (L + 1) + n] = v[m];
  }
}
template <typename R, int L, int NP, int NT>
__device__ inline void zstage_out(const cx<R>* S, cx<R>* __restrict__ base, int t, int n3, int64_t plane,
                                  int np_here) {
  using Z = ZStage<L, NP, NT>;
  const int p = t % NP, n0 = t / NP;
  if (p < np_here)
#pragma unroll
    for (int m = 0; m < Z::MAXIT; ++m) {
      const int n = n0 + m * Z::NSTEP;
      if (n < n3) base[(int64_t)n * plane + p] = S[p * (L + 1) + n];
    }
}

// Fused z pass, one wavefront (or part of one) per pencil: T = L / V <= 64 threads own a pencil,
// so the FFT exchanges only synchronise the wavefront. The block's NP pencils (adjacent k1) are
// loaded and stored through LDS with neighbouring threads on neighbouring pencils (coalesced). One
// LDS row per pencil serves the staging and the exchanges of all three components in turn (a
// third of the LDS of a row per component, so more blocks fit a CU); the staging of each component
// is bracketed by block-wide barriers, the exchanges by wavefront barriers.
template <typename R, int L, int V, int NP>
__global__ __launch_bounds__(NP * L / V) void k_zconv4(cx<R>* __restrict__ buf, int n3, int P1, int P2,
                                                       const cx<R>* __restrict__ spec, const cx<R>* __restrict__ tw,
                                                       const int* __restrict__ order) {
  constexpr int T = L / V;
  constexpr int NT = NP * T;
  constexpr int LP = L + 1;
  constexpr int RAD_LAST = ZRad<L, V>::rad(ZRad<L, V>::nst - 1);
  constexpr int NB_LAST = V / RAD_LAST;
  static_assert(T <= 64, "a pencil must fit one wavefront");
  static_assert(zradices_supported<L, V>(), "last stage radix not handled by the exchange steps");
  __shared__ cx<R> S[NP * LP];
  __shared__ cx<R> tws[ZTw<L, V>::size()];   // per-stage twiddle tables
  const int t = threadIdx.x;
  ztw_fill<R, L, V>(tws, tw, t, NT);
  const int k2 = order[2 * blockIdx.x];
  const int k10 = order[2 * blockIdx.x + 1] * NP;
  const int64_t plane = (int64_t)P1 * P2, comp = plane * n3;
  cx<R>* base = buf + (int64_t)k2 * P1 + k10;
  const int np_here = P1 - k10;
  // staging loads of all three components in flight together: element (c, n, p), pencils fastest
  cx<R> sv[3][ZStage<L, NP, NT>::MAXIT];
  zstage_load<R, L, NP, NT>(sv, base, t, n3, plane, comp, np_here);
  const int p = t / T, j = t % T;
  const int k1 = k10 + p;
  const bool valid = k1 < P1;
  cx<R>* Sp = S + p * LP;
  cx<R> H[3][V];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();   // every pencil has read the previous component from its row
    zstage_put<R, L, NP, NT>(S, sv[c], t, n3);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int n = j + T * q;
      H[c][q] = (2 * q < V && n < n3) ? Sp[n] : cx<R>{0, 0};
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    zsync<true>();   // this pencil's row is free: its previous reads have completed
    zfft_c<R, L, V, true>(Sp, H[c], j, tws);
  }
  {
    const int S1 = P1 / 2 + 1, S3 = L / 2 + 1;
    const int f1 = k1 <= P1 / 2 ? k1 : P1 - k1;
    const int f2 = k2 <= P2 / 2 ? k2 : P2 - k2;
    const R s1 = k1 <= P1 / 2 ? (R)1 : (R)-1;
    const R s2 = k2 <= P2 / 2 ? (R)1 : (R)-1;
    const cx<R>* sp = spec + (valid ? 6 * ((int64_t)f2 * S1 + f1) * S3 : 0);
#pragma unroll
    for (int i = 0; i < NB_LAST; ++i)
#pragma unroll
      for (int q = 0; q < RAD_LAST; ++q) {
        const int k3 = j + T * i + (L / RAD_LAST) * q;
        const int f3 = k3 <= L / 2 ? k3 : L - k3;
        const R s3 = k3 <= L / 2 ? (R)1 : (R)-1;
        const cx<R>* rec = sp + f3;
        const cx<R> Txx = rec[0], Tyy = rec[S3], Tzz = rec[2 * S3];
        const cx<R> Txy = (s1 * s2) * rec[3 * S3];
        const cx<R> Txz = (s1 * s3) * rec[4 * S3];
        const cx<R> Tyz = (s2 * s3) * rec[5 * S3];
        const int e = i * RAD_LAST + q;
        const cx<R> x = H[0][e], y = H[1][e], z = H[2][e];
        H[0][e] = Txx * x + Txy * y + Txz * z;
        H[1][e] = Txy * x + Tyy * y + Tyz * z;
        H[2][e] = Txz * x + Tyz * y + Tzz * z;
        // FP64: keep the spectral loads of one frequency at a time (fewer live registers)
        if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
      }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    zsync<true>();
    zfft_c<R, L, V, false>(Sp, H[c], j, tws);
  }
  // outputs one component at a time: each pencil writes its row, the block writes the rows back
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == 0)
      zsync<true>();   // every exchange of this pencil is read before the outputs overwrite its row
    else
      __syncthreads();   // the previous component's rows are written back
#pragma unroll
    for (int q = 0; q < V / 2; ++q) {
      const int n = j + T * q;
      if (n < n3) Sp[n] = H[c][q];
    }
    __syncthreads();
    zstage_out<R, L, NP, NT>(S, base + c * comp, t, n3, plane, np_here);
  }
}

// z-pass configuration per precision (k_zconv4): the smallest number V of values per thread (a
// pencil must also fit one wavefront, T = L / V <= 64), the threads per block, and the LDS per block
// (one staging row per pencil, and the twiddles). Measured at 2 mm (L = 256) and 1 mm (L = 512):
// FP64 with four values per thread, complex64 with eight; at L = 512 four pencils per block beat
// two.
#ifndef ZCONV_VMIN64
#define ZCONV_VMIN64 4
#endif
#ifndef ZCONV_VMIN32
#define ZCONV_VMIN32 8
#endif
#ifndef ZCONV_THREADS
#define ZCONV_THREADS 256
#endif
#ifndef ZCONV_LDS_CAP
#define ZCONV_LDS_CAP 110000
#endif
constexpr int zconv_v(int L, bool fp64) {
  const int vmin = fp64 ? ZCONV_VMIN64 : ZCONV_VMIN32;
  return L / vmin > 64 ? L / 64 : vmin;
}
// entries of the per-stage twiddle tables of a length-L transform with radix V stages (ZTw)
constexpr int ztw_size(int L, int V) {
  int lgL = 0, lgV = 0;
  for (int x = L; x > 1; x >>= 1) ++lgL;
  for (int x = V; x > 1; x >>= 1) ++lgV;
  const int nst = (lgL + lgV - 1) / lgV;
  int rads[16] = {};
  int r = 1;
  for (int i = 0; i + 1 < nst; ++i) {
    rads[i] = V;
    r *= V;
  }
  rads[nst - 1] = L / r;
  int tot = 0, ls = 1;
  for (int s = 0; s + 1 < nst; ++s) tot += (ls *= rads[s]);
  ls = 1;
  for (int u = 0; u + 1 < nst; ++u) tot += (ls *= rads[nst - 1 - u]);
  return tot;
}
static_assert(ztw_size(64, 4) == ZTw<64, 4>::size() && ztw_size(128, 4) == ZTw<128, 4>::size() &&
                  ztw_size(256, 4) == ZTw<256, 4>::size() && ztw_size(512, 8) == ZTw<512, 8>::size() &&
                  ztw_size(1024, 16) == ZTw<1024, 16>::size() && ztw_size(128, 8) == ZTw<128, 8>::size(),
              "twiddle table sizes");
// pencils per block for V values per thread: the thread target, then halved until the staging
// and twiddles fit the LDS budget
constexpr int zconv_np_for(int L, int V, bool fp64) {
  int np = ZCONV_THREADS / (L / V);
  if (np < 1) np = 1;
  const int elem = fp64 ? 16 : 8;
  const int tws = ztw_size(L, V);
  while (np > 1 && (np * (L + 1) + tws) * elem > ZCONV_LDS_CAP) np /= 2;
  return np;
}
// The z-pass candidates the autotuner times at setup (ZCONV_NCAND per length and precision):
// 0 the measured default; 1 half the pencils per block (smaller blocks, more of them); 2 twice the
// values per thread (one fewer exchange for some lengths, more registers), when that keeps at
// least eight threads per pencil.
constexpr int ZCONV_NCAND = 3;
constexpr int zconv_cand_v(int L, bool fp64, int c) {
  const int v0 = zconv_v(L, fp64);
  return (c == 2 && 2 * v0 <= 16 && L / (2 * v0) >= 8) ? 2 * v0 : v0;
}
constexpr int zconv_cand_np(int L, bool fp64, int c) {
  const int v = zconv_cand_v(L, fp64, c);
  const int np = zconv_np_for(L, v, fp64);
  return (c == 1 && np > 1) ? np / 2 : np;
}
constexpr bool zconv_cand_ok(int L, bool fp64, int c) {
  if (c == 0) return true;
  if (c == 1) return zconv_np_for(L, zconv_v(L, fp64), fp64) > 1;
  return zconv_cand_v(L, fp64, 2) != zconv_v(L, fp64);
}

template <int L> struct Split;
template <> struct Split<8> { static constexpr int A = 4, B = 2; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };
template <> struct Split<32> { static constexpr int A = 8, B = 4; };
template <> struct Split<64> { static constexpr int A = 8, B = 8; };
template <> struct Split<128> { static constexpr int A = 16, B = 8; };
template <> struct Split<256> { static constexpr int A = 16, B = 16; };
template <> struct Split<512> { static constexpr int A = 32, B = 16; };
template <> struct Split<1024> { static constexpr int A = 32, B = 32; };
template <typename R, int A> static constexpr int fft2_np() {
  return (sizeof(R) == 8 ? 128 : 256) / A;
}

// ---------------------------------------------------------------------------------------------
// host-side dispatch over the FFT length
template <typename R> static constexpr int zconv_tp(int L) {
  // one component of TP pencils in LDS (<= 33 KB); 3 x TP*L/256 values per thread in registers
  return sizeof(R) == 8 ? (L <= 128 ? 16 : (L <= 256 ? 8 : (L <= 512 ? 4 : 2)))
                        : (L <= 256 ? 16 : (L <= 512 ? 8 : 4));
}

#define VSIE_FFT_SWITCH(L_, BODY)                                 \
  switch (L_) {                                                   \
    case 8: { constexpr int LL = 8; BODY; } break;                \
    case 16: { constexpr int LL = 16; BODY; } break;              \
    case 32: { constexpr int LL = 32; BODY; } break;              \
    case 64: { constexpr int LL = 64; BODY; } break;              \
    case 128: { constexpr int LL = 128; BODY; } break;            \
    case 256: { constexpr int LL = 256; BODY; } break;            \
    case 512: { constexpr int LL = 512; BODY; } break;            \
    case 1024: { constexpr int LL = 1024; BODY; } break;          \
    default: throw Error(VSIE_E_GRID, "unsupported FFT length");  \
  }

template <typename R>
void fft_rows(hipStream_t st, int L, bool fwd, const cx<R>* in, cx<R>* out, int n_in, int n_out, int64_t in_row,
              int64_t out_row, int64_t nrows, const cx<R>* tw) {
  VSIE_FFT_SWITCH(L, {
    constexpr int A = Split<LL>::A;
    constexpr int B = Split<LL>::B;
    constexpr int NP = (sizeof(R) == 8 ? 128 : 256) / A;
    dim3 grid((unsigned)((nrows + NP - 1) / NP));
    if (fwd)
      hipLaunchKernelGGL((k_fft2<R, A, B, NP, true, false>), grid, dim3(NP * A), 0, st, in, out, n_in, n_out, 1, 1, 0,
                         in_row, out_row, nrows, tw, GridSrc<R>{});
    else
      hipLaunchKernelGGL((k_fft2<R, A, B, NP, false, false>), grid, dim3(NP * A), 0, st, in, out, n_in, n_out, 1, 1, 0,
                         in_row, out_row, nrows, tw, GridSrc<R>{});
  });
}

template <typename R>
void fft_rows_grid(hipStream_t st, int L, const cx<R>* xb, const cx<R>* xn, BodyMask mask, const int* vox2row,
                   const uint8_t* rowhas, const int* rowptr, const int* rowrwg, const R* roww, int nprojrows,
                   cx<R>* projv, const GridDims& g, cx<R>* out, const cx<R>* tw) {
  if (g.Ne >= ((int64_t)1 << 31)) throw Error(VSIE_E_GRID, "extended grid of 2^31 or more voxels");
  const bool proj = xn && vox2row && rowhas && nprojrows > 0;
  if (proj)
    hipLaunchKernelGGL(k_proj_rows<R>, dim3((nprojrows + 63) / 64), dim3(256), 0, st, rowptr, rowrwg, roww, xn,
                       nprojrows, projv);
  const GridSrc<R> gs{xb, mask.vox, mask.runs, proj ? vox2row : nullptr, rowhas, projv, g};
  const int64_t nrows = 3LL * g.ne3 * g.ne2;
  VSIE_FFT_SWITCH(L, {
    constexpr int A = Split<LL>::A;
    constexpr int B = Split<LL>::B;
    constexpr int NP = (sizeof(R) == 8 ? 128 : 256) / A;
    dim3 grid((unsigned)((nrows + NP - 1) / NP));
    hipLaunchKernelGGL((k_fft2<R, A, B, NP, true, false, true>), grid, dim3(NP * A), 0, st, nullptr, out, g.ne1, L,
                       1, 1, 0, 0, (int64_t)L, nrows, tw, gs);
  });
}

template <typename R>
void fft_strided(hipStream_t st, int L, bool fwd, const cx<R>* in, cx<R>* out, int n_in, int n_out, int64_t in_stride,
                 int64_t out_stride, int n_lo, int64_t n_hi, int64_t in_hi, int64_t out_hi, const cx<R>* tw) {
  VSIE_FFT_SWITCH(L, {
    constexpr int A = Split<LL>::A;
    constexpr int B = Split<LL>::B;
    constexpr int NP = (sizeof(R) == 8 ? 128 : 256) / A;
    dim3 grid((unsigned)(n_hi * ((n_lo + NP - 1) / NP)));
    if (fwd)
      hipLaunchKernelGGL((k_fft2<R, A, B, NP, true, true>), grid, dim3(NP * A), 0, st, in, out, n_in, n_out, in_stride,
                         out_stride, n_lo, in_hi, out_hi, 0, tw, GridSrc<R>{});
    else
      hipLaunchKernelGGL((k_fft2<R, A, B, NP, false, true>), grid, dim3(NP * A), 0, st, in, out, n_in, n_out, in_stride,
                         out_stride, n_lo, in_hi, out_hi, 0, tw, GridSrc<R>{});
  });
}

int zconv_pencils(int L, bool fp64, int cand) {
  if (L < 64 || L > 1024 || cand < 0 || cand >= ZCONV_NCAND) return 0;
  int np = 0;
  VSIE_FFT_SWITCH(L, {
    if (fp64) {
      if (cand == 0) np = zconv_cand_np(LL, true, 0);
      else if (cand == 1) np = zconv_cand_np(LL, true, 1);
      else np = zconv_cand_np(LL, true, 2);
    } else {
      if (cand == 0) np = zconv_cand_np(LL, false, 0);
      else if (cand == 1) np = zconv_cand_np(LL, false, 1);
      else np = zconv_cand_np(LL, false, 2);
    }
  });
  return np;
}
bool zconv_candidate(int L, bool fp64, int cand) {
  if (L < 64 || L > 1024 || cand < 0 || cand >= ZCONV_NCAND) return false;
  bool ok = false;
  VSIE_FFT_SWITCH(L, {
    if (cand == 0) ok = true;
    else if (cand == 1) ok = zconv_cand_ok(LL, fp64, 1);
    else ok = zconv_cand_ok(LL, fp64, 2);
  });
  return ok;
}
void zconv_shape(int L, bool fp64, int cand, int* v, int* np) {
  *v = 0;
  *np = 0;
  if (!zconv_candidate(L, fp64, cand)) return;
  VSIE_FFT_SWITCH(L, {
    if (cand == 0) *v = zconv_cand_v(LL, fp64, 0);
    else if (cand == 1) *v = zconv_cand_v(LL, fp64, 1);
    else *v = zconv_cand_v(LL, fp64, 2);
  });
  *np = zconv_pencils(L, fp64, cand);
}

std::vector<int> zconv_order(int L, int P1, int P2, bool fp64, int cand) {
  // Blocks that share spectral records (k2 and P2 - k2; k1 tiles t and TL - 1 - t) and input
  // cache lines (neighbouring tiles t, t + 1) form groups of up to eight. Workgroups are handed
  // to the eight XCDs round-robin, so the members of a full group are placed eight positions
  // apart: they run on one XCD, one after another, and share its L2.
  const int NP = zconv_pencils(L, fp64, cand);
  std::vector<int> ord;
  if (NP == 0) return ord;
  const int TL = (P1 + NP - 1) / NP;
  std::vector<std::vector<std::pair<int, int>>> groups;
  std::vector<char> seen((size_t)TL, 0);
  for (int f2 = 0; f2 <= P2 / 2; ++f2) {
    std::vector<int> k2s = {f2};
    if (f2 != 0 && 2 * f2 != P2) k2s.push_back(P2 - f2);
    std::fill(seen.begin(), seen.end(), 0);
    for (int t = 0; t < TL; ++t) {
      if (seen[t]) continue;
      std::vector<int> ts;
      for (int u : {t, t + 1, TL - 1 - t, TL - 2 - t})
        if (u >= 0 && u < TL && !seen[u]) {
          seen[u] = 1;
          ts.push_back(u);
        }
      std::vector<std::pair<int, int>> g;
      for (int k2 : k2s)
        for (int u : ts) g.push_back({k2, u});
      groups.push_back(g);
    }
  }
  const size_t full = 8;
  std::vector<const std::vector<std::pair<int, int>>*> big, rest;
  for (const auto& g : groups) (g.size() == full ? big : rest).push_back(&g);
  ord.reserve(2 * (size_t)P2 * TL);
  const size_t nchunk = big.size() / 8;
  for (size_t c = 0; c < nchunk; ++c)
    for (size_t m = 0; m < full; ++m)
      for (size_t j = 0; j < 8; ++j) {
        const auto& e = (*big[c * 8 + j])[m];
        ord.push_back(e.first);
        ord.push_back(e.second);
      }
  for (size_t i = nchunk * 8; i < big.size(); ++i) rest.push_back(big[i]);
  for (const auto* g : rest)
    for (const auto& e : *g) {
      ord.push_back(e.first);
      ord.push_back(e.second);
    }
  return ord;
}

template <typename R, int LL, int C>
static void zconv_launch(hipStream_t st, cx<R>* buf, int n3, int P1, int P2, const cx<R>* spec, const cx<R>* tw,
                         const int* order) {
  constexpr bool F64 = sizeof(R) == 8;
  if constexpr (zconv_cand_ok(LL, F64, C)) {
    constexpr int V = zconv_cand_v(LL, F64, C);
    constexpr int NP = zconv_cand_np(LL, F64, C);
    dim3 grid((unsigned)(P2 * ((P1 + NP - 1) / NP)));
    hipLaunchKernelGGL((k_zconv4<R, LL, V, NP>), grid, dim3(NP * LL / V), 0, st, buf, n3, P1, P2, spec, tw, order);
  } else {
    throw Error(VSIE_E_ARG, "z-pass candidate not available for this length");
  }
}

template <typename R>
void fft_z_conv(hipStream_t st, int L, cx<R>* buf, int n3, int P1, int P2, const cx<R>* spec, const cx<R>* tw,
                const int* order, int cand) {
  // register-staged Stockham transform: V values per thread and component, one pencil per group
  if (L >= 64 && L <= 1024) {
    if (!order) throw Error(VSIE_E_STATE, "z-pass block order missing");
    VSIE_FFT_SWITCH(L, {
      if constexpr (LL >= 64) {
        if (cand == 0) (zconv_launch<R, LL, 0>)(st, buf, n3, P1, P2, spec, tw, order);
        else if (cand == 1) (zconv_launch<R, LL, 1>)(st, buf, n3, P1, P2, spec, tw, order);
        else if (cand == 2) (zconv_launch<R, LL, 2>)(st, buf, n3, P1, P2, spec, tw, order);
        else throw Error(VSIE_E_ARG, "z-pass candidate out of range");
      }
    });
    return;
  }
  VSIE_FFT_SWITCH(L, {
    constexpr int TP = zconv_tp<R>(LL);
    dim3 grid((unsigned)(P2 * ((P1 + TP - 1) / TP)));
    hipLaunchKernelGGL((k_fft_z_conv<R, LL, TP>), grid, dim3(256), 0, st, buf, n3, P1, P2, spec, tw);
  });
}

template void fft_rows<double>(hipStream_t, int, bool, const cxd*, cxd*, int, int, int64_t, int64_t, int64_t, const cxd*);
template void fft_rows<float>(hipStream_t, int, bool, const cxf*, cxf*, int, int, int64_t, int64_t, int64_t, const cxf*);
template void fft_rows_grid<double>(hipStream_t, int, const cxd*, const cxd*, BodyMask, const int*,
                                    const uint8_t*, const int*, const int*, const double*, int, cxd*, const GridDims&,
                                    cxd*, const cxd*);
template void fft_rows_grid<float>(hipStream_t, int, const cxf*, const cxf*, BodyMask, const int*,
                                   const uint8_t*, const int*, const int*, const float*, int, cxf*, const GridDims&,
                                   cxf*, const cxf*);
template void fft_strided<double>(hipStream_t, int, bool, const cxd*, cxd*, int, int, int64_t, int64_t, int, int64_t,
                                  int64_t, int64_t, const cxd*);
template void fft_strided<float>(hipStream_t, int, bool, const cxf*, cxf*, int, int, int64_t, int64_t, int, int64_t,
                                 int64_t, int64_t, const cxf*);
template void fft_z_conv<double>(hipStream_t, int, cxd*, int, int, int, const cxd*, const cxd*, const int*, int);
template void fft_z_conv<float>(hipStream_t, int, cxf*, int, int, int, const cxf*, const cxf*, const int*, int);

// =============================================================================================
// Matvec kernels
// =============================================================================================

// body rows: tissue y = h^3/chi x + (T * x) ; air y = x
template <typename R>
__global__ void k_body_out(const cx<R>* __restrict__ xb, const cx<R>* __restrict__ E, const cx<R>* __restrict__ dvchi,
                           const uint8_t* __restrict__ mask, cx<R>* __restrict__ yb, GridDims g) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.nv) return;
  int i1 = (int)(p % g.n1), i2 = (int)((p / g.n1) % g.n2), i3 = (int)(p / ((int64_t)g.n1 * g.n2));
  int64_t v = (i1 + g.ob1) + (int64_t)g.ne1 * ((i2 + g.ob2) + (int64_t)g.ne2 * (i3 + g.ob3));
  if (mask[p]) {
    cx<R> d = dvchi[p];
    for (int a = 0; a < 3; ++a) yb[a * g.nv + p] = d * xb[a * g.nv + p] + E[a * g.Ne + v];
  } else {
    for (int a = 0; a < 3; ++a) yb[a * g.nv + p] = xb[a * g.nv + p];
  }
}

// pFFT interpolation (W^T): one wavefront per near RWG
template <typename R>
__global__ __launch_bounds__(64) void k_pfft_gather(const R* __restrict__ W, const int* __restrict__ base,
                                                    const cx<R>* __restrict__ E, cx<R>* __restrict__ yn, GridDims g) {
  const int n = blockIdx.x;
  const int t = threadIdx.x;
  const int b1 = base[3 * n], b2 = base[3 * n + 1], b3 = base[3 * n + 2];
  cx<R> acc = {0, 0};
  for (int e = t; e < 375; e += 64) {
    int a = e / 125, j = e % 125;
    int j1 = j % 5, j2 = (j / 5) % 5, j3 = j / 25;
    int64_t v = (b1 + j1) + (int64_t)g.ne1 * ((b2 + j2) + (int64_t)g.ne2 * (b3 + j3));
    acc += W[(int64_t)n * 375 + e] * E[a * g.Ne + v];
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.re += __shfl_down(acc.re, off, 64);
    acc.im += __shfl_down(acc.im, off, 64);
  }
  if (t == 0) yn[n] = acc;
}

// y[rowid[r]] += sum_e val[e] x[col[e]]  (rows unique); 16 lanes per row, shuffle reduction
template <typename R>
__global__ __launch_bounds__(256) void k_csr_add(const int* __restrict__ rowid, const int* __restrict__ rowptr,
                                                 const int* __restrict__ col, const cx<R>* __restrict__ val,
                                                 const cx<R>* __restrict__ x, cx<R>* __restrict__ y, int nrows) {
  const int r = blockIdx.x * 16 + threadIdx.x / 16;
  const int lane = threadIdx.x % 16;
  cx<R> acc = {0, 0};
  if (r < nrows)
    for (int e = rowptr[r] + lane; e < rowptr[r + 1]; e += 16) acc += val[e] * x[col[e]];
  for (int off = 8; off > 0; off >>= 1) {
    acc.re += __shfl_down(acc.re, off, 16);
    acc.im += __shfl_down(acc.im, off, 16);
  }
  if (r < nrows && lane == 0) y[rowid[r]] += acc;
}

// Low-rank factors are stored rank-major on the device: A[l][i], l < K (<= 256), i < M, so every
// rank vector is contiguous.
// part[ch][l] = sum_{i in chunk ch} op(A[l][i]) x[i], op = conj if CONJ
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_lr_t_partial(const cx<R>* __restrict__ A, const cx<R>* __restrict__ x,
                                                      int64_t M, int K, int64_t chunk, cx<R>* __restrict__ part) {
  __shared__ R rr[4], ri[4];
  const int l = blockIdx.y, ch = blockIdx.x;
  const cx<R>* a = A + (int64_t)l * M;
  const int64_t i0 = ch * chunk, i1 = i0 + chunk < M ? i0 + chunk : M;
  cx<R> acc = {0, 0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += CONJ ? mul_conj_a(a[i], x[i]) : a[i] * x[i];
  for (int off = 32; off > 0; off >>= 1) {
    acc.re += __shfl_down(acc.re, off, 64);
    acc.im += __shfl_down(acc.im, off, 64);
  }
  if (threadIdx.x % 64 == 0) {
    rr[threadIdx.x / 64] = acc.re;
    ri[threadIdx.x / 64] = acc.im;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[(int64_t)ch * K + l] = cx<R>{(rr[0] + rr[1]) + (rr[2] + rr[3]), (ri[0] + ri[1]) + (ri[2] + ri[3])};
}

// y[i] += sum_l op(A[l][i]) t[l]; a block covers 64 rows with four wavefronts splitting the ranks
template <typename R, bool CONJ>
__global__ __launch_bounds__(256) void k_lr_n_add(const cx<R>* __restrict__ A, const cx<R>* __restrict__ t,
                                                  int64_t M, int K, cx<R>* __restrict__ y) {
  __shared__ cx<R> ts[256];
  __shared__ R rr[4][64], ri[4][64];
  for (int l = threadIdx.x; l < K; l += 256) ts[l] = t[l];
  __syncthreads();
  const int row = threadIdx.x % 64, sl = threadIdx.x / 64;
  const int64_t i = (int64_t)blockIdx.x * 64 + row;
  cx<R> acc = {0, 0};
  if (i < M)
    for (int l = sl; l < K; l += 4) {
      cx<R> a = A[(int64_t)l * M + i];
      acc += CONJ ? mul_conj_a(a, ts[l]) : a * ts[l];
    }
  rr[sl][row] = acc.re;
  ri[sl][row] = acc.im;
  __syncthreads();
  if (sl == 0 && i < M)
    y[i] += cx<R>{(rr[0][row] + rr[1][row]) + (rr[2][row] + rr[3][row]),
                  (ri[0][row] + ri[1][row]) + (ri[2][row] + ri[3][row])};
}

// Both products with a row-major block of rows in one pass over it: for every row l (flattened
// over up to three blocks A_b [nrows_b][m], row r of block b at l = off_b + r) the partial sums
// part[blk][l] = sum over the workgroup's columns i of op(A[l][i]) x[i], and the column sums
// ypart[g][i] = sum over row group g of op(A[l][i]) s[l] (op = conj if CONJ; y += sum_g ypart[g]
// afterwards). Each element is read once. A workgroup of 16 wavefronts covers DUAL_COLS columns
// (DUAL_CPL per lane, 64 apart, so that a row's lane sums cover several columns before they are
// combined across the wavefront) and one of DUAL_RG row groups: wavefront w of group g takes rows
// 16 g + w + 16 DUAL_RG k. s holds at most DUAL_MAXROWS entries.
constexpr int DUAL_CPL = 4;
constexpr int DUAL_COLS = 64 * DUAL_CPL;
constexpr int DUAL_RG = 2;
constexpr int DUAL_MAXROWS = 384;
template <typename R> struct DualRows {
  const cx<R>* A[3];
  int nrows[3];
  int off[3];
  int nblock;
};
template <typename R, bool CONJ>
__global__ __launch_bounds__(1024) void k_dual_rows(DualRows<R> D, const cx<R>* __restrict__ x,
                                                    const cx<R>* __restrict__ s, int64_t m,
                                                    cx<R>* __restrict__ ypart, cx<R>* __restrict__ part, int pstride) {
  __shared__ cx<R> sv[DUAL_MAXROWS];
  __shared__ R yr[16][DUAL_COLS], yi[16][DUAL_COLS];
  const int t = threadIdx.x;
  for (int l = t; l < pstride; l += 1024) sv[l] = s[l];
  __syncthreads();
  const int lane = t % 64, w = t / 64, g = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * DUAL_COLS + lane;
  cx<R> xv[DUAL_CPL], ya[DUAL_CPL];
#pragma unroll
  for (int q = 0; q < DUAL_CPL; ++q) {
    const int64_t i = i0 + 64 * q;
    xv[q] = i < m ? x[i] : cx<R>{0, 0};
    ya[q] = cx<R>{0, 0};
  }
  int nr = 0;
  for (int b = 0; b < D.nblock; ++b) nr += D.nrows[b];
  for (int r = 16 * g + w; r < nr; r += 16 * DUAL_RG) {
    int b = 0, rr = r;
    while (b + 1 < D.nblock && rr >= D.nrows[b]) rr -= D.nrows[b++];
    const int l = D.off[b] + rr;
    const cx<R>* a = D.A[b] + (int64_t)rr * m;
    const cx<R> sl = sv[l];
    cx<R> av[DUAL_CPL];
#pragma unroll
    for (int q = 0; q < DUAL_CPL; ++q) {
      const int64_t i = i0 + 64 * q;
      av[q] = i < m ? a[i] : cx<R>{0, 0};
    }
    cx<R> pr = {0, 0};
#pragma unroll
    for (int q = 0; q < DUAL_CPL; ++q) {
      if (CONJ) {
        pr += mul_conj_a(av[q], xv[q]);
        ya[q] += mul_conj_a(av[q], sl);
      } else {
        pr += av[q] * xv[q];
        ya[q] += av[q] * sl;
      }
    }
    R re = pr.re, im = pr.im;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o, 64);
      im += __shfl_xor(im, o, 64);
    }
    if (lane == 0) part[(int64_t)blockIdx.x * pstride + l] = cx<R>{re, im};
  }
#pragma unroll
  for (int q = 0; q < DUAL_CPL; ++q) {
    yr[w][lane + 64 * q] = ya[q].re;
    yi[w][lane + 64 * q] = ya[q].im;
  }
  __syncthreads();
  if (t < DUAL_COLS) {
    const int64_t i = (int64_t)blockIdx.x * DUAL_COLS + t;
    if (i < m) {
      cx<R> acc = {0, 0};
#pragma unroll
      for (int q = 0; q < 16; ++q) acc += cx<R>{yr[q][t], yi[q][t]};
      ypart[(int64_t)g * m + i] = acc;
    }
  }
}

// y[i] += sum_g ypart[g][i], g < DUAL_RG
template <typename R>
__global__ __launch_bounds__(256) void k_dual_finish(const cx<R>* __restrict__ ypart, int64_t m, cx<R>* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  cx<R> acc = y[i];
#pragma unroll
  for (int g = 0; g < DUAL_RG; ++g) acc += ypart[(int64_t)g * m + i];
  y[i] = acc;
}


// out[l] = sum_b part[b][l]: one block per column, tree reduction
template <typename R>
__global__ __launch_bounds__(256) void k_sum_partials(const cx<R>* __restrict__ part, int nblk, int K,
                                                      cx<R>* __restrict__ out) {
  __shared__ R rr[256], ri[256];
  const int l = blockIdx.x;
  cx<R> acc = {0, 0};
  for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(int64_t)b * K + l];
  rr[threadIdx.x] = acc.re;
  ri[threadIdx.x] = acc.im;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) {
      rr[threadIdx.x] += rr[threadIdx.x + s2];
      ri[threadIdx.x] += ri[threadIdx.x + s2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[l] = cx<R>{rr[0], ri[0]};
}

// the launches of one pass: partial sums of part (nblk x pstride) into out, y += column sums
template <typename R, bool CONJ>
static void launch_dual(hipStream_t st, const DualRows<R>& D, const cx<R>* x, const cx<R>* s, int64_t m, cx<R>* y,
                        cx<R>* ypart, cx<R>* part, int pstride, cx<R>* out) {
  const unsigned nb = (unsigned)((m + DUAL_COLS - 1) / DUAL_COLS);
  hipLaunchKernelGGL((k_dual_rows<R, CONJ>), dim3(nb, DUAL_RG), dim3(1024), 0, st, D, x, s, m, ypart, part, pstride);
  hipLaunchKernelGGL(k_dual_finish<R>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, ypart, m, y);
  hipLaunchKernelGGL(k_sum_partials<R>, dim3(pstride), dim3(256), 0, st, part, (int)nb, pstride, out);
}
int64_t dual_work_elems(int64_t m) { return ((m + DUAL_COLS - 1) / DUAL_COLS) * DUAL_MAXROWS + DUAL_RG * m; }

// one block per row: out[row] = sum_j A[row][j] x[j]  (dense GEMV, row-major, write)
template <typename R>
__global__ __launch_bounds__(256) void k_gemv_rows(const cx<R>* __restrict__ A, const cx<R>* __restrict__ x,
                                                   int64_t ncol, cx<R>* __restrict__ out, int accumulate) {
  __shared__ R rr[256], ri[256];
  const int64_t row = blockIdx.x;
  const cx<R>* a = A + row * ncol;
  cx<R> acc = {0, 0};
  for (int64_t j = threadIdx.x; j < ncol; j += 256) acc += a[j] * x[j];
  rr[threadIdx.x] = acc.re;
  ri[threadIdx.x] = acc.im;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rr[threadIdx.x] += rr[threadIdx.x + s];
      ri[threadIdx.x] += ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cx<R> v = {rr[0], ri[0]};
    if (accumulate) out[row] += v;
    else out[row] = v;
  }
}

// Symmetric far block from its upper-triangle tiles: each tile (I, J) is read once (blocks step
// over the tiles, one per block at the default grid) and yields both the row sums Z_IJ x_J and
// (for I < J) the column sums Z_IJ^T x_I.
// Thread (rg, cg): column lane cg owns columns cg + 32 c, c < 4, so each load instruction of a
// half-wavefront reads 512 contiguous bytes of one row; 8 row groups of 16 rows. Row sums reduce
// across the 32 column lanes by shuffles; column sums across row groups by one shuffle and LDS.
template <typename R>
__global__ __launch_bounds__(256) void k_symv_tiles(const cx<R>* __restrict__ Zp, const int* __restrict__ tiles,
                                                    const cx<R>* __restrict__ x, int m, int64_t ntiles,
                                                    cx<R>* __restrict__ part) {
  __shared__ R cr[4][SYM_TB], ci[4][SYM_TB];
  __shared__ cx<R> xs[SYM_TB];
  const int cg = threadIdx.x % 32, rg = threadIdx.x / 32;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int I = tiles[2 * t], J = tiles[2 * t + 1];
    const cx<R>* Z = Zp + t * (int64_t)SYM_TB * SYM_TB;
    if (threadIdx.x < SYM_TB) {
      int mm = I * SYM_TB + threadIdx.x;
      xs[threadIdx.x] = mm < m ? x[mm] : cx<R>{0, 0};
    }
    cx<R> xJ[4], ca[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int n = J * SYM_TB + cg + 32 * c;
      xJ[c] = n < m ? x[n] : cx<R>{0, 0};
      ca[c] = {0, 0};
    }
    __syncthreads();
    cx<R>* out = part + t * 2 * SYM_TB;
#pragma unroll 4
    for (int r = 0; r < 16; ++r) {
      const int row = rg * 16 + r;
      const cx<R>* zr = Z + (int64_t)row * SYM_TB + cg;
      const cx<R> xi = xs[row];
      cx<R> rd = {0, 0};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const cx<R> z = ld_stream(zr + 32 * c);   // each tile is read once per product
        rd += z * xJ[c];
        ca[c] += z * xi;
      }
      for (int off = 16; off > 0; off >>= 1) {
        rd.re += __shfl_xor(rd.re, off, 32);
        rd.im += __shfl_xor(rd.im, off, 32);
      }
      if (cg == 0) out[row] = rd;
    }
    if (I != J) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        ca[c].re += __shfl_xor(ca[c].re, 32, 64);
        ca[c].im += __shfl_xor(ca[c].im, 32, 64);
      }
      const int wave = threadIdx.x / 64;
      if ((threadIdx.x % 64) < 32)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          cr[wave][cg + 32 * c] = ca[c].re;
          ci[wave][cg + 32 * c] = ca[c].im;
        }
      __syncthreads();
      if (threadIdx.x < SYM_TB) {
        int c = threadIdx.x;
        out[SYM_TB + c] = cx<R>{cr[0][c] + cr[1][c] + cr[2][c] + cr[3][c], ci[0][c] + ci[1][c] + ci[2][c] + ci[3][c]};
      }
    }
    __syncthreads();   // xs, cr and ci are rewritten by the next tile
  }
}

// y[i] = sum_{J >= I} rowpart(I, J)[i] + sum_{J < I} colpart(J, I)[i], I = i / SYM_TB; a block
// covers 64 outputs with four wavefronts taking every fourth J (fixed order)
template <typename R>
__global__ __launch_bounds__(256) void k_symv_reduce(const cx<R>* __restrict__ part, int T, int m,
                                                     cx<R>* __restrict__ y, int accumulate) {
  __shared__ R rr[4][64], ri[4][64];
  const int o = threadIdx.x % 64, sl = threadIdx.x / 64;
  const int i = blockIdx.x * 64 + o;
  cx<R> acc = {0, 0};
  if (i < m) {
    const int I = i / SYM_TB, li = i % SYM_TB;
    for (int J = sl; J < T; J += 4) {
      if (J < I) {
        const int64_t t = (int64_t)J * T - (int64_t)J * (J - 1) / 2 + (I - J);
        acc += part[t * 2 * SYM_TB + SYM_TB + li];
      } else {
        const int64_t t = (int64_t)I * T - (int64_t)I * (I - 1) / 2 + (J - I);
        acc += part[t * 2 * SYM_TB + li];
      }
    }
  }
  rr[sl][o] = acc.re;
  ri[sl][o] = acc.im;
  __syncthreads();
  if (sl == 0 && i < m) {
    const cx<R> v = {(rr[0][o] + rr[1][o]) + (rr[2][o] + rr[3][o]), (ri[0][o] + ri[1][o]) + (ri[2][o] + ri[3][o])};
    if (accumulate) y[i] += v;
    else y[i] = v;
  }
}

// ---------------------------------------------------------------------------------------------
// 64 x 64 output tile per block of 256 threads on the matrix cores: each wavefront owns a 32 x 32
// quadrant as 2 x 2 tiles of the 16 x 16 x 4 MFMA (FP64: v_mfma_f64_16x16x4f64, FP32:
// v_mfma_f32_16x16x4f32); K is staged through LDS in chunks of 16, tile loaders walking each
// operand's unit-stride dimension.
// A complex product is four real MFMAs (re re, -im im into the real part; re im, im re into the
// imaginary part). Operand lane layout: A[row l % 16][k l / 16], B[k l / 16][col l % 16]; result
// lane l, register v: FP64 row l / 16 + 4 v, FP32 row 4 (l / 16) + v, column l % 16 (both
// checked on the device). Columns run along lanes, so C is best given with unit column stride.
typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename R> struct Mfma16;
template <> struct Mfma16<double> {
  typedef dvec4 V;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct Mfma16<float> {
  typedef fvec4 V;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * (lane / 16) + v; }
};

template <typename R>
__global__ __launch_bounds__(256) void k_zgemm_mfma(GemmSet<R> S) {
  using MM = Mfma16<R>;
  using V = typename MM::V;
  __shared__ cx<R> As[64][17];
  __shared__ cx<R> Bs[16][65];
  int z = blockIdx.z, pi = 0;
  while (pi + 1 < S.nprob && z >= S.nbatch[pi]) {
    z -= S.nbatch[pi];
    ++pi;
  }
  const GemmArgs<R>& g = pi == 0 ? S.g[0] : (pi == 1 ? S.g[1] : S.g[2]);
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  int K = g.K;
  if (g.ktot > 0) K = (int)(g.ktot - (int64_t)z * g.K < g.K ? g.ktot - (int64_t)z * g.K : g.K);
  if (i0 >= g.M || j0 >= g.N || K <= 0) return;
  const bool a_rowfast = g.sac != 1 && g.sar == 1;
  const bool b_rowfast = g.sbc != 1 && g.sbr == 1;
  const cx<R>* A = g.A + z * g.sab;
  const cx<R>* B = g.B + z * g.sbb;
  const uint8_t* mB = g.maskB ? g.maskB + z * g.sbb : nullptr;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wm = (wave / 2) * 32, wn = (wave % 2) * 32;
  const int li = lane % 16, lk = lane / 16;
  V cr[2][2], ci[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      cr[u][v] = V{0, 0, 0, 0};
      ci[u][v] = V{0, 0, 0, 0};
    }
  // FP64: the next K chunk is loaded into registers while the current one is multiplied from LDS
  // (FP32 keeps load-then-store: the extra registers would cost it a wavefront per SIMD)
  constexpr bool prefetch = sizeof(R) == 8;
  cx<R> pa[4], pb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = a_rowfast ? e % 64 : e / 16, c = a_rowfast ? e / 64 : e % 16;
      const int i = i0 + r, k = k0 + c;
      pa[q] = (i < g.M && k < K) ? A[i * g.sar + k * g.sac] : cx<R>{0, 0};
      const int rb = b_rowfast ? e % 16 : e / 64, cb = b_rowfast ? e / 16 : e % 64;
      const int kk = k0 + rb, j = j0 + cb;
      cx<R> v = {0, 0};
      if (kk < K && j < g.N) {
        const int64_t idx = kk * g.sbr + j * g.sbc;
        v = B[idx];
        if (mB && !mB[idx]) v = cx<R>{0, 0};
      }
      pb[q] = v;
    }
  };
  if (prefetch) load(0);
  for (int k0 = 0; k0 < K; k0 += 16) {
    if (!prefetch) load(k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[a_rowfast ? e % 64 : e / 16][a_rowfast ? e / 64 : e % 16] = pa[q];
      Bs[b_rowfast ? e % 16 : e / 64][b_rowfast ? e / 16 : e % 64] = pb[q];
    }
    __syncthreads();
    if (prefetch && k0 + 16 < K) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      cx<R> a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) a[u] = As[wm + 16 * u + li][ks + lk];
#pragma unroll
      for (int v = 0; v < 2; ++v) b[v] = Bs[ks + lk][wn + 16 * v + li];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          cr[u][v] = MM::mma(a[u].re, b[v].re, cr[u][v]);
          cr[u][v] = MM::mma(-a[u].im, b[v].im, cr[u][v]);
          ci[u][v] = MM::mma(a[u].re, b[v].im, ci[u][v]);
          ci[u][v] = MM::mma(a[u].im, b[v].re, ci[u][v]);
        }
    }
    __syncthreads();
  }
  cx<R>* C = g.C + z * g.scb;
  const uint8_t* mC = g.maskC;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + wm + 16 * u + MM::row(lane, e), j = j0 + wn + 16 * v + li;
        if (i >= g.M || j >= g.N) continue;
        const cx<R> val = g.negate ? cx<R>{-cr[u][v][e], -ci[u][v][e]} : cx<R>{cr[u][v][e], ci[u][v][e]};
        const int64_t idx = i * g.scr + j * g.scc;
        if (mC) {
          if (mC[idx]) C[idx] += val;
        } else if (g.accumulate) {
          C[idx] += val;
        } else {
          C[idx] = val;
        }
      }
}

template <typename R> void launch_zgemm(hipStream_t st, const GemmSet<R>& S) {
  int mx = 0, nx = 0, nz = 0;
  for (int p = 0; p < S.nprob; ++p) {
    mx = std::max(mx, S.g[p].M);
    nx = std::max(nx, S.g[p].N);
    nz += S.nbatch[p];
  }
  if (mx <= 0 || nx <= 0 || nz <= 0) return;
  hipLaunchKernelGGL(k_zgemm_mfma<R>, dim3((nx + 63) / 64, (mx + 63) / 64, nz), dim3(256), 0, st, S);
}
template void launch_zgemm<double>(hipStream_t, const GemmSet<double>&);
template void launch_zgemm<float>(hipStream_t, const GemmSet<float>&);

// The far-block tile pass for up to 16 right-hand sides on the matrix cores (column b of x at
// x + b ldx, its partials at part + b ldp). For a tile (I, J) the row sums Z X_J and the column
// sums Z^T X_I are complex products of the 128 x 128 tile with 128 x nrhs slices of x, i.e. GEMMs
// whose output columns are the right-hand sides: the 16 x 16 x 4 MFMA takes them along its
// 16 output columns, and the reductions over the tile happen inside the matrix core. The tile
// streams through LDS in slabs of 32 rows. Each of the four waves takes one 16-row block of the
// slab for the row sums over one half of the columns (the halves are added through LDS), and two
// 16-column blocks for the column sums, accumulated over all slabs in registers.
template <typename R>
__global__ __launch_bounds__(256) void k_symv_multi(const cx<R>* __restrict__ Zp, const int* __restrict__ tiles,
                                                    const cx<R>* __restrict__ x, int64_t ldx, int m, int nrhs,
                                                    int64_t ntiles, cx<R>* __restrict__ part, int64_t ldp) {
  using MM = Mfma16<R>;
  using V = typename MM::V;
  constexpr int SL = 32, LD = SYM_TB + 1;
  __shared__ cx<R> zs[SL * LD];
  __shared__ cx<R> red[2][16][16];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int li = lane % 16, lk = lane / 16;
  const int kh = w / 2, rb = w % 2;   // column half and row block of this wave's row sums
  const bool live = li < nrhs;
  for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
    const int I = tiles[2 * tt], J = tiles[2 * tt + 1];
    const cx<R>* Z = Zp + tt * (int64_t)SYM_TB * SYM_TB;
    cx<R>* out = part + tt * 2 * SYM_TB;
    cx<R> bj[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int mm = J * SYM_TB + kh * 64 + 4 * q + lk;
      bj[q] = (live && mm < m) ? x[li * ldx + mm] : cx<R>{0, 0};
    }
    V ccr[2], cci[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      ccr[cb] = V{0, 0, 0, 0};
      cci[cb] = V{0, 0, 0, 0};
    }
    for (int s = 0; s < SYM_TB / SL; ++s) {
      __syncthreads();   // the previous slab and its row-sum exchange are consumed
      for (int e = threadIdx.x; e < SL * SYM_TB; e += 256) {
        const int r = e / SYM_TB, c = e % SYM_TB;
        zs[r * LD + c] = ld_stream(Z + (int64_t)(s * SL + r) * SYM_TB + c);   // each tile is read once
      }
      __syncthreads();
      V rr = V{0, 0, 0, 0}, ri = V{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const cx<R> a = zs[(rb * 16 + li) * LD + kh * 64 + 4 * q + lk];
        rr = MM::mma(a.re, bj[q].re, rr);
        rr = MM::mma(-a.im, bj[q].im, rr);
        ri = MM::mma(a.re, bj[q].im, ri);
        ri = MM::mma(a.im, bj[q].re, ri);
      }
      if (kh == 1)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[rb][MM::row(lane, v)][li] = cx<R>{rr[v], ri[v]};
      if (I != J) {
#pragma unroll
        for (int q = 0; q < SL / 4; ++q) {
          const int mm = I * SYM_TB + s * SL + 4 * q + lk;
          const cx<R> b = (live && mm < m) ? x[li * ldx + mm] : cx<R>{0, 0};
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            const cx<R> a = zs[(4 * q + lk) * LD + (2 * w + cb) * 16 + li];
            ccr[cb] = MM::mma(a.re, b.re, ccr[cb]);
            ccr[cb] = MM::mma(-a.im, b.im, ccr[cb]);
            cci[cb] = MM::mma(a.re, b.im, cci[cb]);
            cci[cb] = MM::mma(a.im, b.re, cci[cb]);
          }
        }
      }
      __syncthreads();
      if (kh == 0 && live)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = MM::row(lane, v);
          out[li * ldp + s * SL + rb * 16 + row] = cx<R>{rr[v], ri[v]} + red[rb][row][li];
        }
    }
    if (I != J && live)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[li * ldp + SYM_TB + (2 * w + cb) * 16 + MM::row(lane, v)] = cx<R>{ccr[cb][v], cci[cb][v]};
  }
}

// s2[c][j2][i3] = sum_b part[c][b][j2][i3], b < nb_c = ceil(r1_c n2 / kc) (split-K reduction of
// the transpose contraction over (j1, i2)); a block covers 32 outputs with 8 slices over b
template <typename R>
__global__ __launch_bounds__(256) void k_tt_ksum(TTDesc<R> T, const cx<R>* __restrict__ part, int kc, int n2, int n3,
                                                 cx<R>* __restrict__ s2) {
  __shared__ R rr[8][32], ri[8][32];
  const int c = blockIdx.y;
  const int o = threadIdx.x % 32, sl = threadIdx.x / 32;
  const int id = blockIdx.x * 32 + o;
  const bool live = id < T.r2[c] * n3;
  const int nb = (T.r1[c] * n2 + kc - 1) / kc;
  cx<R> acc = {0, 0};
  if (live) {
    const cx<R>* p = part + (int64_t)c * TT_KBATCH * TT_RMAX * n3 + id;
    for (int b = sl; b < nb; b += 8) acc += p[(int64_t)b * TT_RMAX * n3];
  }
  rr[sl][o] = acc.re;
  ri[sl][o] = acc.im;
  __syncthreads();
  if (sl == 0 && live) {
    cx<R> s = {0, 0};
#pragma unroll
    for (int q = 0; q < 8; ++q) s += cx<R>{rr[q][o], ri[q][o]};
    s2[(int64_t)c * TT_RMAX * n3 + id] = s;
  }
}

// ---------------------------------------------------------------------------------------------
// Tensor-train far coupling (eqs. (16)-(19)). Cores row-major: G1[i1][j1], G2[j1][i2][j2],
// G3[j2][i3][j3], G4[j3][i4]. The body index is i1 + n1 i2 + n1 n2 i3 = i1 + n1 row with
// row = i2 + n2 i3. Intermediates per component, contracted one core at a time so that the work
// on the body-sized vectors costs r1 products per voxel (the smallest rank):
//   forward   t4[j3] -> t3[j2][i3] -> U[i3][j1][i2] = sum_j2 G2[j1][i2][j2] t3[j2][i3]
//             -> y_b[i1 + n1 row] += mask * sum_j1 G1[i1][j1] U[i3][j1][i2]
//   transpose T1[i3][j1][i2] = sum_i1 G1[i1][j1] mask x_b[i1 + n1 row]
//             -> S2[j2][i3] = sum_(j1, i2) G2[j1][i2][j2] T1[i3][j1][i2] -> s3[j3] -> y_f[i4]

// T1 on the matrix cores: a wavefront owns 16 rows (the MFMA's columns) and a 16-wide tile of j1
// (its rows), K = i1 in steps of 4 over the union of the 16 rows' tissue runs; operands straight
// from memory (x_b is read only inside the runs, G1 is a few KB and stays in cache). t1 points at
// component 0; components are t1_cs apart.
template <typename R>
__global__ __launch_bounds__(256) void k_tt_t1(TTDesc<R> T, const cx<R>* __restrict__ xb, BodyMask mask, int n1,
                                               int n2, int rows, int64_t nv, cx<R>* __restrict__ t1, int64_t t1_cs) {
  using MM = Mfma16<R>;
  using V = typename MM::V;
  const int c = blockIdx.y;
  const int r1 = T.r1[c];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int row0 = (blockIdx.x * 4 + wave) * 16;
  if (row0 >= rows) return;   // the whole wavefront leaves
  const int li = lane % 16, lk = lane / 16;
  const int row = row0 + li;
  const bool rv = row < rows;
  const cx<R>* xr = xb + (int64_t)c * nv + (int64_t)(rv ? row : 0) * n1;
  const uint8_t* mr = mask.vox + (int64_t)(rv ? row : 0) * n1;
  const int2 run = rv ? mask.runs[row] : int2{0, 0};
  const bool holes = run.x < 0;
  const int lo = holes ? ~run.x : run.x, hi = run.y;
  // K range of the wavefront: the union of its rows' runs
  int klo = hi > lo ? lo : n1, khi = hi > lo ? hi : 0;
  for (int o = 8; o > 0; o >>= 1) {
    klo = min(klo, __shfl_xor(klo, o, 16));
    khi = max(khi, __shfl_xor(khi, o, 16));
  }
  klo &= ~3;
  const cx<R>* g1 = T.G1[c];
  const int i3 = row / n2, i2 = row - (row / n2) * n2;
  cx<R>* out = t1 + (int64_t)c * t1_cs + (int64_t)i3 * r1 * n2 + i2;
  constexpr int KB = 8;   // K-steps whose operands are loaded together (loads in flight)
  for (int jt = 0; jt < r1; jt += 16) {
    const int ja = jt + li;   // the A row this lane supplies
    V dr = V{0, 0, 0, 0}, di = V{0, 0, 0, 0};
    for (int kb = klo; kb < khi; kb += 4 * KB) {
      cx<R> a[KB], b[KB];
      uint8_t mk[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const int i1 = kb + 4 * q + lk;
        const bool in = i1 < khi;
        const bool tin = rv && i1 >= lo && i1 < hi;   // inside this row's run (hence i1 < n1)
        a[q] = (ja < r1 && in) ? g1[(int64_t)i1 * r1 + ja] : cx<R>{0, 0};
        b[q] = tin ? xr[i1] : cx<R>{0, 0};
        mk[q] = (tin && holes) ? mr[i1] : (uint8_t)tin;
      }
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const cx<R> bb = mk[q] ? b[q] : cx<R>{0, 0};
        dr = MM::mma(a[q].re, bb.re, dr);
        dr = MM::mma(-a[q].im, bb.im, dr);
        di = MM::mma(a[q].re, bb.im, di);
        di = MM::mma(a[q].im, bb.re, di);
      }
    }
    if (rv)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j1 = jt + MM::row(lane, v);
        if (j1 < r1) out[(int64_t)j1 * n2] = cx<R>{dr[v], di[v]};
      }
  }
}

// y_b[c][i1 + n1 row] += mask * sum_j1 G1[c][i1][j1] U[c][i3][j1][i2], one voxel per thread
// (consecutive threads on consecutive voxels: coalesced read-modify-write of y_b)
template <typename R>
__global__ __launch_bounds__(256) void k_tt_yb(TTDesc<R> T, const cx<R>* __restrict__ u, int64_t u_cs,
                                               const uint8_t* __restrict__ mask, int n1, int n2, int nv,
                                               cx<R>* __restrict__ yb) {
  const int c = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nv || !mask[e]) return;
  const unsigned row = (unsigned)e / (unsigned)n1;
  const int i1 = e - (int)row * n1;
  const unsigned i3 = row / (unsigned)n2;
  const int i2 = (int)row - (int)i3 * n2;
  const int r1 = T.r1[c];
  const cx<R>* g = T.G1[c] + (int64_t)i1 * r1;
  const cx<R>* uc = u + (int64_t)c * u_cs + (int64_t)i3 * r1 * n2 + i2;
  cx<R> acc = {0, 0};
  for (int j1 = 0; j1 < r1; ++j1) acc += g[j1] * uc[(int64_t)j1 * n2];
  yb[(int64_t)c * nv + e] += acc;
}

// t3[c][row] = sum_j3 G3[row][j3] t4v[c][j3] over rows (j2, i3) of G3; t4 staged in LDS; 16 lanes
// per row read it contiguously, 16 rows per block
template <typename R>
__global__ __launch_bounds__(256) void k_tt_f3(TTDesc<R> T, const cx<R>* __restrict__ t4v, int n3,
                                               cx<R>* __restrict__ t3) {
  __shared__ cx<R> t4[TT_RMAX];
  const int c = blockIdx.y;
  const int r2 = T.r2[c], r3 = T.r3[c];
  for (int j3 = threadIdx.x; j3 < r3; j3 += 256) t4[j3] = t4v[c * TT_RMAX + j3];
  __syncthreads();
  const int row = blockIdx.x * 16 + threadIdx.x / 16;
  const int lane = threadIdx.x % 16;
  cx<R> acc = {0, 0};
  if (row < r2 * n3) {
    const cx<R>* g = T.G3[c] + (int64_t)row * r3;
    for (int j3 = lane; j3 < r3; j3 += 16) acc += g[j3] * t4[j3];
  }
  for (int off = 8; off > 0; off >>= 1) {
    acc.re += __shfl_xor(acc.re, off, 16);
    acc.im += __shfl_xor(acc.im, off, 16);
  }
  if (lane == 0 && row < r2 * n3) t3[(int64_t)c * TT_RMAX * n3 + row] = acc;
}

// partial sums of s3[c][j3] = sum_k G3[k][j3] S2[c][k] over rows k = (j2, i3) of G3, TT_KROWS rows
// per block: part[blk][c TT_RMAX + j3] (zero for j3 >= r3)
constexpr int TT_KROWS = 16;
template <typename R>
__global__ __launch_bounds__(256) void k_ttT_3(TTDesc<R> T, const cx<R>* __restrict__ s2, int n3,
                                               cx<R>* __restrict__ part) {
  __shared__ R rr[4][TT_RMAX], ri[4][TT_RMAX];
  const int c = blockIdx.y;
  const int r2 = T.r2[c], r3 = T.r3[c];
  const int K = r2 * n3;
  const int lane = threadIdx.x % 64, sl = threadIdx.x / 64;
  const int k0 = blockIdx.x * TT_KROWS;
  const cx<R>* sv = s2 + (int64_t)c * TT_RMAX * n3;
  for (int j3 = lane; j3 < TT_RMAX; j3 += 64) {
    cx<R> acc = {0, 0};
    if (j3 < r3)
#pragma unroll
      for (int q = 0; q < TT_KROWS / 4; ++q) {
        const int k = k0 + sl + 4 * q;
        if (k < K) acc += T.G3[c][(int64_t)k * r3 + j3] * sv[k];
      }
    rr[sl][j3] = acc.re;
    ri[sl][j3] = acc.im;
  }
  __syncthreads();
  for (int j3 = threadIdx.x; j3 < TT_RMAX; j3 += 256)
    part[(int64_t)blockIdx.x * 3 * TT_RMAX + c * TT_RMAX + j3] =
        cx<R>{(rr[0][j3] + rr[1][j3]) + (rr[2][j3] + rr[3][j3]), (ri[0][j3] + ri[1][j3]) + (ri[2][j3] + ri[3][j3])};
}

// =============================================================================================
// Solver helpers (FP64 Arnoldi) and conversions
// =============================================================================================

// partial sums of V[i]^H w for i < nvec: part[blk][nvec]. Grid-stride over rows; vectors in
// groups of eight per block reduction (w is re-read per group from cache).
__global__ __launch_bounds__(256) void k_multidot_partial(const cxd* __restrict__ V, int64_t ld, int nvec,
                                                          const cxd* __restrict__ w, int64_t n, int64_t s1, int64_t s2,
                                                          int with_norm, cxd* __restrict__ part) {
  constexpr int G = 8;
  __shared__ double rr[G + 3][4], ri[G + 3][4];
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int K = nvec + (with_norm ? 3 : 0);
  for (int i0 = 0; i0 < nvec || (i0 == 0 && with_norm); i0 += G) {
    const int g = nvec - i0 < G ? nvec - i0 : G;
    const bool nrm = with_norm && i0 == 0;
    cxd acc[G];
    double sq[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < G; ++q) acc[q] = cxd{0, 0};
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += stride) {
      const cxd wr = w[r];
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (q < g) acc[q] += mul_conj_a(V[(int64_t)(i0 + q) * ld + r], wr);
      if (nrm) sq[r < s1 ? 0 : (r < s2 ? 1 : 2)] += wr.re * wr.re + wr.im * wr.im;
    }
#pragma unroll
    for (int q = 0; q < G + 3; ++q) {
      double re = q < G ? acc[q].re : sq[q - G], im = q < G ? acc[q].im : 0.0;
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
      }
      if (lane == 0) {
        rr[q][wave] = re;
        ri[q][wave] = im;
      }
    }
    __syncthreads();
    const int t = threadIdx.x;
    const auto sum4 = [&](int q) {
      return cxd{(rr[q][0] + rr[q][1]) + (rr[q][2] + rr[q][3]), (ri[q][0] + ri[q][1]) + (ri[q][2] + ri[q][3])};
    };
    if (t < g) part[(int64_t)blockIdx.x * K + i0 + t] = sum4(t);
    if (nrm && t >= 64 && t < 67) part[(int64_t)blockIdx.x * K + nvec + (t - 64)] = sum4(G + t - 64);
    __syncthreads();
  }
}

// w -= sum_i h[i] V[i], and per-block partial sums of |w|^2 over [0, s1), [s1, s2), [s2, n)
// after the update (part[blk][3], real parts)
__global__ __launch_bounds__(256) void k_multiaxpy_norm(const cxd* __restrict__ V, int64_t ld, int nvec,
                                                        const cxd* __restrict__ h, cxd* __restrict__ w, int64_t n,
                                                        int64_t s1, int64_t s2, cxd* __restrict__ part) {
  __shared__ cxd hs[1024];
  __shared__ double red[3][4];
  for (int i = threadIdx.x; i < nvec; i += 256) hs[i] = h[i];
  __syncthreads();
  double sq[3] = {0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += stride) {
    cxd acc = w[r];
    for (int i = 0; i < nvec; ++i) acc -= hs[i] * V[(int64_t)i * ld + r];
    w[r] = acc;
    sq[r < s1 ? 0 : (r < s2 ? 1 : 2)] += acc.re * acc.re + acc.im * acc.im;
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int s = 0; s < 3; ++s) {
    double v = sq[s];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[s][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3)
    part[(int64_t)blockIdx.x * 3 + threadIdx.x] =
        cxd{(red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]), 0.0};
}

// x += sum_i y[i] V[i]
__global__ void k_combine_add(const cxd* __restrict__ V, int64_t ld, int nvec, const cxd* __restrict__ y,
                              cxd* __restrict__ x, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  cxd acc = x[r];
  for (int i = 0; i < nvec; ++i) acc += y[i] * V[(int64_t)i * ld + r];
  x[r] = acc;
}

__global__ void k_scale_copy(const cxd* __restrict__ a, double s, cxd* __restrict__ b, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = s * a[r];
}

__global__ void k_sub(const cxd* __restrict__ a, const cxd* __restrict__ b, cxd* __restrict__ c, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) c[r] = a[r] - b[r];
}

__global__ void k_add(cxd* __restrict__ a, const cxd* __restrict__ b, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) a[r] += b[r];
}

__global__ void k_d2f(const cxd* __restrict__ a, cxf* __restrict__ b, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = cxf{(float)a[r].re, (float)a[r].im};
}

__global__ void k_f2d(const cxf* __restrict__ a, cxd* __restrict__ b, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) b[r] = cxd{(double)a[r].re, (double)a[r].im};
}

// partial sums of |a|^2 over segments [s0, s1) for three segments at once: part[blk][4]
__global__ __launch_bounds__(256) void k_norm_partial(const cxd* __restrict__ a, int64_t n, int64_t s1, int64_t s2,
                                                      double* __restrict__ part) {
  __shared__ double red[4][256];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  double acc[3] = {0, 0, 0};
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    double v = a[r].re * a[r].re + a[r].im * a[r].im;
    int seg = r < s1 ? 0 : (r < s2 ? 1 : 2);
    acc[seg] += v;
  }
  for (int s = 0; s < 3; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[(int64_t)blockIdx.x * 3 + q] = red[q][0];
}

// port right-hand side
template <typename R>
__global__ void k_scatter_rhs(const int* __restrict__ idx, const double* __restrict__ val_re,
                              const double* __restrict__ val_im, int ne, cx<R>* __restrict__ b) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) b[idx[e]] = cx<R>{(R)val_re[e], (R)val_im[e]};
}

// ---------------------------------------------------------------------------------------------
// explicit instantiations and host launchers
template <typename R> void launch_body_out(hipStream_t st, const cx<R>* xb, const cx<R>* E, const cx<R>* dvchi,
                                           const uint8_t* mask, cx<R>* yb, const GridDims& g) {
  hipLaunchKernelGGL(k_body_out<R>, dim3((unsigned)((g.nv + 255) / 256)), dim3(256), 0, st, xb, E, dvchi, mask, yb, g);
}
template <typename R> void launch_pfft_gather(hipStream_t st, const R* W, const int* base, const cx<R>* E, cx<R>* yn,
                                              int mn, const GridDims& g) {
  if (mn > 0) hipLaunchKernelGGL(k_pfft_gather<R>, dim3(mn), dim3(64), 0, st, W, base, E, yn, g);
}
template <typename R> void launch_csr_add(hipStream_t st, const int* rowid, const int* rowptr, const int* col,
                                          const cx<R>* val, const cx<R>* x, cx<R>* y, int nrows) {
  if (nrows > 0) hipLaunchKernelGGL(k_csr_add<R>, dim3((nrows + 15) / 16), dim3(256), 0, st, rowid, rowptr, col, val, x, y, nrows);
}
template <typename R> void launch_lr_t(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* x, int64_t M, int K,
                                       cx<R>* part, int max_chunks, cx<R>* out) {
  if (K <= 0) return;
  if (K > 256) throw Error(VSIE_E_ARG, "low-rank factor wider than 256 columns");
  int64_t chunk = 2048;
  while ((M + chunk - 1) / chunk > max_chunks) chunk *= 2;
  const int nch = (int)((M + chunk - 1) / chunk);
  if (nch == 0) return;
  if (conj)
    hipLaunchKernelGGL((k_lr_t_partial<R, true>), dim3(nch, K), dim3(256), 0, st, A, x, M, K, chunk, part);
  else
    hipLaunchKernelGGL((k_lr_t_partial<R, false>), dim3(nch, K), dim3(256), 0, st, A, x, M, K, chunk, part);
  hipLaunchKernelGGL(k_sum_partials<R>, dim3(K), dim3(256), 0, st, part, nch, K, out);
}
template <typename R> void launch_lr_dual(hipStream_t st, const cx<R>* V, int K, int64_t M, const cx<R>* x,
                                          const cx<R>* s, cx<R>* y, cx<R>* work, cx<R>* out) {
  if (K <= 0 || M <= 0) return;
  if (K > 256) throw Error(VSIE_E_ARG, "low-rank factor wider than 256 columns");
  DualRows<R> D{};
  D.nblock = 1;
  D.A[0] = V;
  D.nrows[0] = K;
  cx<R>* ypart = work;
  cx<R>* part = work + DUAL_RG * M;
  launch_dual<R, true>(st, D, x, s, M, y, ypart, part, K, out);
}
int64_t lr_dual_part_elems(int64_t M) { return dual_work_elems(M); }
template <typename R> void launch_lr_n_add(hipStream_t st, bool conj, const cx<R>* A, const cx<R>* t, int64_t M,
                                           int K, cx<R>* y) {
  if (M <= 0 || K <= 0) return;
  const unsigned nb = (unsigned)((M + 63) / 64);
  if (conj)
    hipLaunchKernelGGL((k_lr_n_add<R, true>), dim3(nb), dim3(256), 0, st, A, t, M, K, y);
  else
    hipLaunchKernelGGL((k_lr_n_add<R, false>), dim3(nb), dim3(256), 0, st, A, t, M, K, y);
}
template <typename R> void launch_gemv_rows(hipStream_t st, const cx<R>* A, const cx<R>* x, int64_t nrow, int64_t ncol,
                                            cx<R>* out, int accumulate) {
  if (nrow > 0) hipLaunchKernelGGL(k_gemv_rows<R>, dim3((unsigned)nrow), dim3(256), 0, st, A, x, ncol, out, accumulate);
}
// TT work layout (element offsets fixed by n and m_f): s3 (3 RMAX) | t3 (3 RMAX n3) | s2 (3 RMAX
// n3) | split-K partials (3 KBATCH RMAX n3) | s3 partials (nk3 3 RMAX) | T1 or U (3 components of
// n3 RMAX n2) | G4 pass partial sums and column sums (dual_work_elems) | t4 (3 RMAX)
struct TTWork {
  int n1, n2, n3, mf, nk3, rmax1, rmax2, rmax3, kc2;
  int64_t nv, o_t3, o_s2, o_kpart, o_s3part, o_t1, o_t4part, o_t4, t1_cs, total;
};
static TTWork tt_offsets(const int n[3], int mf) {
  TTWork w{};
  w.n1 = n[0];
  w.n2 = n[1];
  w.n3 = n[2];
  w.nv = (int64_t)n[0] * n[1] * n[2];
  w.mf = mf;
  const int nk3max = (TT_RMAX * w.n3 + TT_KROWS - 1) / TT_KROWS;
  w.o_t3 = 3LL * TT_RMAX;
  w.o_s2 = w.o_t3 + 3LL * TT_RMAX * w.n3;
  w.o_kpart = w.o_s2 + 3LL * TT_RMAX * w.n3;
  w.o_s3part = w.o_kpart + 3LL * TT_KBATCH * TT_RMAX * w.n3;
  w.o_t1 = w.o_s3part + 3LL * TT_RMAX * nk3max;
  w.t1_cs = (int64_t)TT_RMAX * w.n2 * w.n3;
  w.o_t4part = w.o_t1 + 3 * w.t1_cs;
  w.o_t4 = w.o_t4part + dual_work_elems(std::max(mf, 1));
  w.total = w.o_t4 + 3LL * TT_RMAX;
  return w;
}
template <typename R> static TTWork tt_layout(const TTDesc<R>& T, const int n[3], int mf) {
  TTWork w = tt_offsets(n, mf);
  w.rmax1 = w.rmax2 = w.rmax3 = 1;
  for (int c = 0; c < 3; ++c) {
    w.rmax1 = std::max(w.rmax1, T.r1[c]);
    w.rmax2 = std::max(w.rmax2, T.r2[c]);
    w.rmax3 = std::max(w.rmax3, T.r3[c]);
  }
  w.nk3 = (w.rmax2 * w.n3 + TT_KROWS - 1) / TT_KROWS;
  // split-K chunk of the (j1, i2) contraction: a multiple of 16 giving at most KBATCH batches
  const int k2 = w.rmax1 * w.n2;
  w.kc2 = 16 * (((k2 + TT_KBATCH - 1) / TT_KBATCH + 15) / 16);
  if (w.nv >= ((int64_t)1 << 31)) throw Error(VSIE_E_GRID, "TT coupling of a body of 2^31 or more voxels");
  return w;
}

// The TT coupling up to its accumulation into y_b: the transpose chain from x_b to s3
// (eqs. (18)-(19)), then one pass over G4 for y_f += sum_c G4^T s3 and the forward G4 x_f
// (eq. (16)), then G3 into t3 (eq. (17)). y_f must already hold the rest of its product.
template <typename R> void launch_tt_pre(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf, const cx<R>* xf,
                                         const cx<R>* xb, BodyMask mask, cx<R>* yf, cx<R>* work) {
  const TTWork w = tt_layout(T, n, mf);
  launch_tt_transpose_pre<R>(st, T, n, mf, xb, mask, work);
  const cx<R>* s3 = work;
  cx<R>* t4part = work + w.o_t4part;
  cx<R>* t4 = work + w.o_t4;
  DualRows<R> G{};
  G.nblock = 3;
  for (int c = 0; c < 3; ++c) {
    G.A[c] = T.G4[c];
    G.nrows[c] = T.r3[c];
    G.off[c] = c * TT_RMAX;
  }
  launch_dual<R, false>(st, G, xf, s3, (int64_t)mf, yf, t4part + dual_work_elems(mf) - DUAL_RG * (int64_t)mf,
                        t4part, 3 * TT_RMAX, t4);
  hipLaunchKernelGGL(k_tt_f3<R>, dim3((w.rmax2 * w.n3 + 15) / 16, 3), dim3(256), 0, st, T, t4, w.n3,
                     work + w.o_t3);
}

// The transpose half of launch_tt_pre: s3[c][j3] (at the start of the work buffer) from x_b.
template <typename R> void launch_tt_transpose_pre(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                   const cx<R>* xb, BodyMask mask, cx<R>* work) {
  const TTWork w = tt_layout(T, n, mf);
  cx<R>* s2 = work + w.o_s2;
  cx<R>* kpart = work + w.o_kpart;
  cx<R>* s3part = work + w.o_s3part;
  cx<R>* t1 = work + w.o_t1;
  cx<R>* s3 = work;
  const int rows = w.n2 * w.n3;
  // T1[c][i3][j1][i2] over the first core (x_b read once)
  hipLaunchKernelGGL(k_tt_t1<R>, dim3((rows + 63) / 64, 3), dim3(256), 0, st, T, xb, mask, w.n1, w.n2, rows, w.nv, t1,
                     w.t1_cs);
  // S2(j2, i3) = sum_k G2[k][j2] T1[i3][k], k = (j1, i2), split over k in chunks of kc2
  GemmSet<R> B{};
  B.nprob = 3;
  for (int c = 0; c < 3; ++c) {
    const int ktot = T.r1[c] * w.n2;
    B.g[c] = GemmArgs<R>{T.G2[c], 1, T.r2[c], (int64_t)w.kc2 * T.r2[c], t1 + c * w.t1_cs, 1, ktot, w.kc2,
                         kpart + (int64_t)c * TT_KBATCH * TT_RMAX * w.n3, w.n3, 1, (int64_t)TT_RMAX * w.n3,
                         T.r2[c], w.n3, w.kc2, ktot, nullptr, nullptr, 0, 0};
    B.nbatch[c] = (ktot + w.kc2 - 1) / w.kc2;
  }
  launch_zgemm<R>(st, B);
  hipLaunchKernelGGL(k_tt_ksum<R>, dim3((w.rmax2 * w.n3 + 31) / 32, 3), dim3(256), 0, st, T, kpart, w.kc2, w.n2, w.n3,
                     s2);
  hipLaunchKernelGGL(k_ttT_3<R>, dim3(w.nk3, 3), dim3(256), 0, st, T, s2, w.n3, s3part);
  hipLaunchKernelGGL(k_sum_partials<R>, dim3(3 * TT_RMAX), dim3(256), 0, st, s3part, w.nk3, 3 * TT_RMAX, s3);
}

// Forward chain from given rank-r3 vectors u3[c][j3] (in place of G4 x_f): t3 = G3 u3.
template <typename R> void launch_tt_forward_from(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                  const cx<R>* u3, cx<R>* work) {
  const TTWork w = tt_layout(T, n, mf);
  cx<R>* t3 = work + w.o_t3;
  hipLaunchKernelGGL(k_tt_f3<R>, dim3((w.rmax2 * w.n3 + 15) / 16, 3), dim3(256), 0, st, T, u3, w.n3, t3);
}

// The accumulation into y_b from the work buffer filled by launch_tt_pre.
template <typename R> void launch_tt_post(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                          const uint8_t* mask, cx<R>* yb, cx<R>* work) {
  launch_tt_forward_post<R>(st, T, n, mf, mask, yb, work);
}

// The forward half of launch_tt_post: U = G2 t3, then y_b[c] += mask * G1 U.
template <typename R> void launch_tt_forward_post(hipStream_t st, const TTDesc<R>& T, const int n[3], int mf,
                                                  const uint8_t* mask, cx<R>* yb, cx<R>* work) {
  const TTWork w = tt_layout(T, n, mf);
  const cx<R>* t3 = work + w.o_t3;
  cx<R>* u = work + w.o_t1;
  GemmSet<R> F{};
  F.nprob = 3;
  for (int c = 0; c < 3; ++c) {
    // U(k, i3) = U[c][i3][k], k = (j1, i2): sum_j2 G2[k][j2] t3[j2][i3]
    const int K2 = T.r1[c] * w.n2;
    F.g[c] = GemmArgs<R>{T.G2[c], T.r2[c], 1, 0, t3 + (int64_t)c * TT_RMAX * w.n3, w.n3, 1, 0, u + c * w.t1_cs, 1, K2,
                         0, K2, w.n3, T.r2[c], 0, nullptr, nullptr, 0, 0};
    F.nbatch[c] = 1;
  }
  launch_zgemm<R>(st, F);
  hipLaunchKernelGGL(k_tt_yb<R>, dim3((unsigned)((w.nv + 255) / 256), 3), dim3(256), 0, st, T, u, w.t1_cs, mask, w.n1,
                     w.n2, (int)w.nv, yb);
}
int64_t tt_work_elems(const int n[3], int mf) { return tt_offsets(n, mf).total; }
template <typename R> void launch_symv_tiles(hipStream_t st, const cx<R>* Zp, const int* tiles, int T, const cx<R>* x,
                                             int m, cx<R>* part) {
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  hipLaunchKernelGGL(k_symv_tiles<R>, dim3((unsigned)nt), dim3(256), 0, st, Zp, tiles, x, m, nt, part);
}
template <typename R> void launch_symv_multi(hipStream_t st, const cx<R>* Zp, const int* tiles, int T, const cx<R>* x,
                                             int64_t ldx, int m, int nrhs, cx<R>* part, int64_t ldp) {
  if (nrhs < 1 || nrhs > 16) throw Error(VSIE_E_ARG, "symv_multi takes 1 to 16 right-hand sides");
  const int64_t nt = (int64_t)T * (T + 1) / 2;
  hipLaunchKernelGGL(k_symv_multi<R>, dim3((unsigned)nt), dim3(256), 0, st, Zp, tiles, x, ldx, m, nrhs, nt, part, ldp);
}
template <typename R> void launch_symv_reduce(hipStream_t st, const cx<R>* part, int T, int m, cx<R>* y) {
  hipLaunchKernelGGL(k_symv_reduce<R>, dim3((m + 63) / 64), dim3(256), 0, st, part, T, m, y, 0);
}
template <typename R> void launch_scatter_rhs(hipStream_t st, const int* idx, const double* vre, const double* vim,
                                             int ne, cx<R>* b) {
  if (ne > 0) hipLaunchKernelGGL(k_scatter_rhs<R>, dim3((ne + 255) / 256), dim3(256), 0, st, idx, vre, vim, ne, b);
}

// ---------------------------------------------------------------------------------------------
// Elimination of the far-conductor currents (Schur complement of the dense far block) and the
// block-Jacobi preconditioner of the reduced system, FP64.
//
// The far currents couple to the rest only through low-rank factors: Z_fr x_r = L t(x_r) with
// L = [conj(V) | G4_0^T | G4_1^T | G4_2^T] (m_f x K) and t = [U^T x_n ; s3_0 ; s3_1 ; s3_2], the
// ACA (eq. (12)) and the transpose TT chain (eqs. (18)-(19)). With W = Z_ff^-1 L and
// S = L^T W (K x K), the reduced operator is Z_rr x_r - R^T (S t(x_r)), where R^T injects proxy
// values through the same factors in the forward direction (U p_a into y_n, the forward TT chain
// from p_c into y_b, eqs. (16)-(17)).

// dense row-major m x m copy of a symmetric block held as upper-triangle tiles
__global__ void k_unpack_sym(const cxd* __restrict__ Zp, int T, int m, cxd* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  int I = i / SYM_TB, J = j / SYM_TB, a = i % SYM_TB, b = j % SYM_TB;
  if (I > J) {
    const int t0 = I, t1 = a;
    I = J;
    J = t0;
    a = b;
    b = t1;
  }
  const int64_t t = (int64_t)I * T - (int64_t)I * (I - 1) / 2 + (J - I);
  out[e] = Zp[t * SYM_TB * SYM_TB + a * SYM_TB + b];
}

// upper-triangle tiles (tile list as for the far block) of a dense row-major m x m matrix
__global__ void k_pack_sym(const cxd* __restrict__ X, int m, const int* __restrict__ tiles, int64_t ntiles,
                           cxd* __restrict__ Zp) {
  const int64_t per = (int64_t)SYM_TB * SYM_TB;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntiles * per) return;
  const int64_t t = e / per;
  const int a = (int)((e % per) / SYM_TB), b = (int)(e % SYM_TB);
  const int i = tiles[2 * t] * SYM_TB + a, j = tiles[2 * t + 1] * SYM_TB + b;
  Zp[e] = (i < m && j < m) ? X[(int64_t)i * m + j] : cxd{0, 0};
}

// L[i][l], row-major m_f x K: conj(V[l][i]) for the ka ACA columns, then G4_c[r][i] per component
__global__ void k_build_far_factors(const cxd* __restrict__ V, int ka, TTDesc<double> T, int mf, int K,
                                    cxd* __restrict__ L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mf * K) return;
  const int i = (int)(e / K), l = (int)(e % K);
  cxd v;
  if (l < ka) {
    v = conj(V[(int64_t)l * mf + i]);
  } else {
    int q = l - ka, c = 0;
    while (c < 2 && q >= T.r3[c]) q -= T.r3[c++];
    v = T.G4[c][(int64_t)q * mf + i];
  }
  L[e] = v;
}

// p = sign * S t, t = [ta (ka values) | s3[0][0..r3_0) | s3[1][..] | s3[2][..]] (s3 rows of
// length TT_RMAX); p is scattered the same way into pa and p3. One wavefront per row of S.
constexpr int SCHUR_KMAX = 256 + 3 * TT_RMAX;
template <typename R>
__global__ __launch_bounds__(256) void k_schur_apply(const cx<R>* __restrict__ S, int K, int ka, int r30, int r31,
                                                     int r32, const cx<R>* __restrict__ ta,
                                                     const cx<R>* __restrict__ s3, R sign, cx<R>* __restrict__ pa,
                                                     cx<R>* __restrict__ p3) {
  __shared__ cx<R> t[SCHUR_KMAX];
  for (int l = threadIdx.x; l < K; l += 256) {
    if (l < ka) {
      t[l] = ta[l];
    } else {
      const int q = l - ka;
      const int c = q < r30 ? 0 : (q < r30 + r31 ? 1 : 2);
      const int r = q - (c > 0 ? r30 : 0) - (c > 1 ? r31 : 0);
      t[l] = s3[c * TT_RMAX + r];
    }
  }
  __syncthreads();
  const int row = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (row >= K) return;
  cx<R> acc = {0, 0};
  for (int m = lane; m < K; m += 64) acc += S[(int64_t)row * K + m] * t[m];
  for (int off = 32; off > 0; off >>= 1) {
    acc.re += __shfl_xor(acc.re, off, 64);
    acc.im += __shfl_xor(acc.im, off, 64);
  }
  if (lane != 0) return;
  acc = sign * acc;
  if (row < ka) {
    pa[row] = acc;
  } else {
    const int q = row - ka;
    const int c = q < r30 ? 0 : (q < r30 + r31 ? 1 : 2);
    const int r = q - (c > 0 ? r30 : 0) - (c > 1 ? r31 : 0);
    p3[c * TT_RMAX + r] = acc;
  }
}

// out[l] = sign * t[l] with t laid out as for k_schur_apply (compact proxy vector)
__global__ void k_schur_gather(int K, int ka, int r30, int r31, const cxd* __restrict__ ta,
                               const cxd* __restrict__ s3, double sign, cxd* __restrict__ out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  cxd v;
  if (l < ka) {
    v = ta[l];
  } else {
    const int q = l - ka;
    const int c = q < r30 ? 0 : (q < r30 + r31 ? 1 : 2);
    const int r = q - (c > 0 ? r30 : 0) - (c > 1 ? r31 : 0);
    v = s3[c * TT_RMAX + r];
  }
  out[l] = sign * v;
}

// pa / p3 (layout as in k_schur_apply) = sign * in, in compact (K values)
__global__ void k_schur_scatter(int K, int ka, int r30, int r31, const cxd* __restrict__ in, double sign,
                                cxd* __restrict__ pa, cxd* __restrict__ p3) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= K) return;
  const cxd v = sign * in[l];
  if (l < ka) {
    pa[l] = v;
  } else {
    const int q = l - ka;
    const int c = q < r30 ? 0 : (q < r30 + r31 ? 1 : 2);
    const int r = q - (c > 0 ? r30 : 0) - (c > 1 ? r31 : 0);
    p3[c * TT_RMAX + r] = v;
  }
}

// dst[i] = src[idx[i]] and dst[idx[i]] = src[i]: the unknowns that couple (conductor currents
// and tissue voxels) packed into and out of a compact vector
__global__ void k_gather_idx(const cxd* __restrict__ src, const int* __restrict__ idx, int64_t n, cxd* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}
__global__ void k_scatter_idx(const cxd* __restrict__ src, const int* __restrict__ idx, int64_t n, cxd* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = src[i];
}

// y = d * x elementwise
template <typename R>
__global__ void k_mul_diag(const cx<R>* __restrict__ x, const cx<R>* __restrict__ d, cx<R>* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = d[i] * x[i];
}

// X = identity (n x n, row-major)
__global__ void k_set_identity(cxd* __restrict__ X, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  X[e] = cxd{e / n == e % n ? 1.0 : 0.0, 0.0};
}

void launch_set_identity(hipStream_t st, cxd* X, int n) {
  const int64_t m = (int64_t)n * n;
  if (m > 0) hipLaunchKernelGGL(k_set_identity, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, X, n);
}
void launch_unpack_sym(hipStream_t st, const cxd* Zp, int T, int m, cxd* out) {
  const int64_t n = (int64_t)m * m;
  if (n > 0) hipLaunchKernelGGL(k_unpack_sym, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Zp, T, m, out);
}
void launch_pack_sym(hipStream_t st, const cxd* X, int m, const int* tiles, int64_t ntiles, cxd* Zp) {
  const int64_t n = ntiles * SYM_TB * SYM_TB;
  if (n > 0) hipLaunchKernelGGL(k_pack_sym, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, m, tiles, ntiles, Zp);
}
void launch_build_far_factors(hipStream_t st, const cxd* V, int ka, const TTDesc<double>& T, int mf, int K, cxd* L) {
  const int64_t n = (int64_t)mf * K;
  if (n > 0)
    hipLaunchKernelGGL(k_build_far_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, V, ka, T, mf, K, L);
}
template <typename R>
void launch_schur_apply(hipStream_t st, const cx<R>* S, int K, int ka, const int r3[3], const cx<R>* ta,
                        const cx<R>* s3, R sign, cx<R>* pa, cx<R>* p3) {
  if (K > SCHUR_KMAX) throw Error(VSIE_E_ARG, "more than " + std::to_string(SCHUR_KMAX) + " far-coupling proxies");
  if (K > 0)
    hipLaunchKernelGGL(k_schur_apply<R>, dim3((K + 3) / 4), dim3(256), 0, st, S, K, ka, r3[0], r3[1], r3[2], ta, s3, sign,
                       pa, p3);
}
void launch_schur_gather(hipStream_t st, int K, int ka, const int r3[3], const cxd* ta, const cxd* s3, double sign,
                         cxd* out) {
  if (K > 0) hipLaunchKernelGGL(k_schur_gather, dim3((K + 255) / 256), dim3(256), 0, st, K, ka, r3[0], r3[1], ta, s3, sign, out);
}
void launch_schur_scatter(hipStream_t st, int K, int ka, const int r3[3], const cxd* in, double sign, cxd* pa,
                          cxd* p3) {
  if (K > 0) hipLaunchKernelGGL(k_schur_scatter, dim3((K + 255) / 256), dim3(256), 0, st, K, ka, r3[0], r3[1], in, sign, pa, p3);
}
void launch_gather_idx(hipStream_t st, const cxd* src, const int* idx, int64_t n, cxd* dst) {
  if (n > 0) hipLaunchKernelGGL(k_gather_idx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, idx, n, dst);
}
void launch_scatter_idx(hipStream_t st, const cxd* src, const int* idx, int64_t n, cxd* dst) {
  if (n > 0) hipLaunchKernelGGL(k_scatter_idx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, idx, n, dst);
}
template <typename R> void launch_mul_diag(hipStream_t st, const cx<R>* x, const cx<R>* d, cx<R>* y, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_mul_diag<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, d, y, n);
}
template void launch_schur_apply<double>(hipStream_t, const cxd*, int, int, const int[3], const cxd*, const cxd*,
                                         double, cxd*, cxd*);
template void launch_schur_apply<float>(hipStream_t, const cxf*, int, int, const int[3], const cxf*, const cxf*, float,
                                        cxf*, cxf*);
template void launch_mul_diag<double>(hipStream_t, const cxd*, const cxd*, cxd*, int64_t);
template void launch_mul_diag<float>(hipStream_t, const cxf*, const cxf*, cxf*, int64_t);

#define VSIE_INST(R)                                                                                                  \
  template void launch_body_out<R>(hipStream_t, const cx<R>*, const cx<R>*, const cx<R>*, const uint8_t*, cx<R>*,     \
                                   const GridDims&);                                                                 \
  template void launch_pfft_gather<R>(hipStream_t, const R*, const int*, const cx<R>*, cx<R>*, int, const GridDims&); \
  template void launch_csr_add<R>(hipStream_t, const int*, const int*, const int*, const cx<R>*, const cx<R>*,        \
                                  cx<R>*, int);                                                                      \
  template void launch_lr_t<R>(hipStream_t, bool, const cx<R>*, const cx<R>*, int64_t, int, cx<R>*, int, cx<R>*);      \
  template void launch_lr_n_add<R>(hipStream_t, bool, const cx<R>*, const cx<R>*, int64_t, int, cx<R>*);              \
  template void launch_lr_dual<R>(hipStream_t, const cx<R>*, int, int64_t, const cx<R>*, const cx<R>*, cx<R>*, cx<R>*, \
                                  cx<R>*);                                                                            \
  template void launch_gemv_rows<R>(hipStream_t, const cx<R>*, const cx<R>*, int64_t, int64_t, cx<R>*, int);          \
  template void launch_tt_pre<R>(hipStream_t, const TTDesc<R>&, const int[3], int, const cx<R>*, const cx<R>*,       \
                                 BodyMask, cx<R>*, cx<R>*);                                                           \
  template void launch_tt_post<R>(hipStream_t, const TTDesc<R>&, const int[3], int, const uint8_t*, cx<R>*,           \
                                  cx<R>*);                                                                            \
  template void launch_tt_transpose_pre<R>(hipStream_t, const TTDesc<R>&, const int[3], int, const cx<R>*,          \
                                           BodyMask, cx<R>*);                                                   \
  template void launch_tt_forward_from<R>(hipStream_t, const TTDesc<R>&, const int[3], int, const cx<R>*, cx<R>*); \
  template void launch_tt_forward_post<R>(hipStream_t, const TTDesc<R>&, const int[3], int, const uint8_t*,        \
                                          cx<R>*, cx<R>*);                                                \
  template void launch_scatter_rhs<R>(hipStream_t, const int*, const double*, const double*, int, cx<R>*);         \
  template void launch_symv_tiles<R>(hipStream_t, const cx<R>*, const int*, int, const cx<R>*, int, cx<R>*);      \
  template void launch_symv_reduce<R>(hipStream_t, const cx<R>*, int, int, cx<R>*);                                            \
  template void launch_symv_multi<R>(hipStream_t, const cx<R>*, const int*, int, const cx<R>*, int64_t, int, int, cx<R>*, \
                                     int64_t);
VSIE_INST(double)
VSIE_INST(float)

void launch_generator(hipStream_t st, const GaussTab* gt, const int ne[3], double kappa, const CellRule& cr, cxd* oct) {
  int64_t S = (int64_t)ne[0] * ne[1] * ne[2];
  hipLaunchKernelGGL(k_generator_octant, dim3((unsigned)((S + 63) / 64)), dim3(64), 0, st, gt, ne[0], ne[1], ne[2],
                     kappa, cr, oct);
}
void launch_embed_circulant(hipStream_t st, const cxd* oct, const int ne[3], const int P[3], cxd* full) {
  int64_t PT = (int64_t)P[0] * P[1] * P[2];
  hipLaunchKernelGGL(k_embed_circulant, dim3((unsigned)((PT + 255) / 256)), dim3(256), 0, st, oct, ne[0], ne[1], ne[2],
                     P[0], P[1], P[2], full);
}
template <typename R> void launch_extract_octant(hipStream_t st, const cxd* full, const int P[3], double scale, cx<R>* spec) {
  int64_t SO = (int64_t)(P[0] / 2 + 1) * (P[1] / 2 + 1) * (P[2] / 2 + 1);
  hipLaunchKernelGGL(k_extract_octant<R>, dim3((unsigned)((SO + 255) / 256)), dim3(256), 0, st, full, P[0], P[1], P[2],
                     scale, spec);
}
template void launch_extract_octant<double>(hipStream_t, const cxd*, const int[3], double, cxd*);
template void launch_extract_octant<float>(hipStream_t, const cxd*, const int[3], double, cxf*);

void launch_zcc_dense(hipStream_t st, const RwgDev& A, const RwgDev& B, double k, int64_t row0, int64_t nrows, cxd* out) {
  int64_t tot = nrows * B.m;
  if (tot > 0) hipLaunchKernelGGL(k_zcc_dense, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, st, A, B, k, row0, nrows, out);
}
void launch_zcc_packed(hipStream_t st, const RwgDev& A, double k, const int* tiles, int64_t tile0, int64_t ntiles,
                       cxd* out) {
  int64_t tot = ntiles * SYM_TB * SYM_TB;
  if (tot > 0)
    hipLaunchKernelGGL(k_zcc_packed, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, st, A, k, tiles, tile0, ntiles, out);
}
void launch_zcc_pairs(hipStream_t st, const RwgDev& A, const RwgDev& B, const int* pi, const int* pj, int64_t np,
                      double k, cxd* out) {
  if (np > 0) hipLaunchKernelGGL(k_zcc_pairs, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, st, A, B, pi, pj, np, k, out);
}
void launch_pfft_wtw(hipStream_t st, const double* W, const int* base, const cxd* oct, const int ne[3], const int* pm,
                     const int* pn, int64_t np, cxd* out) {
  if (np > 0) hipLaunchKernelGGL(k_pfft_wtw_pairs, dim3((unsigned)np), dim3(256), 0, st, W, base, oct, ne[0], ne[1], ne[2], pm, pn, out);
}
void launch_pfft_tw_voxels(hipStream_t st, const double* W, const int* base, const cxd* oct, const int ne[3],
                           const int* vox, const int* pn, int64_t np, cxd* out) {
  if (np > 0)
    hipLaunchKernelGGL(k_pfft_tw_voxels, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, st, W, base, oct, ne[0], ne[1],
                       ne[2], vox, pn, np, out);
}
void launch_zbc_near(hipStream_t st, const RwgDev& B, const double* centres, const int* pn, int64_t np, double h,
                     double k, cxd* out) {
  if (np > 0)
    hipLaunchKernelGGL(k_zbc_near_pairs, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, st, B, centres, pn, np, h, k, out);
}

void launch_multidot(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* w, int64_t n, int64_t s1,
                     int64_t s2, int with_norm, cxd* part, int nblk) {
  hipLaunchKernelGGL(k_multidot_partial, dim3(nblk), dim3(256), 0, st, V, ld, nvec, w, n, s1, s2, with_norm, part);
}
void launch_sum_partials(hipStream_t st, const cxd* part, int nblk, int K, cxd* out) {
  if (K > 0) hipLaunchKernelGGL(k_sum_partials<double>, dim3(K), dim3(256), 0, st, part, nblk, K, out);
}
void launch_multiaxpy_norm(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* h, cxd* w, int64_t n,
                          int64_t s1, int64_t s2, cxd* part, int nblk) {
  if (nvec > 1024) throw Error(VSIE_E_ARG, "Krylov basis wider than 1024");
  hipLaunchKernelGGL(k_multiaxpy_norm, dim3(nblk), dim3(256), 0, st, V, ld, nvec, h, w, n, s1, s2, part);
}
void launch_combine_add(hipStream_t st, const cxd* V, int64_t ld, int nvec, const cxd* y, cxd* x, int64_t n) {
  hipLaunchKernelGGL(k_combine_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, V, ld, nvec, y, x, n);
}
void launch_scale_copy(hipStream_t st, const cxd* a, double s, cxd* b, int64_t n) {
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, s, b, n);
}
void launch_sub(hipStream_t st, const cxd* a, const cxd* b, cxd* c, int64_t n) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, c, n);
}
void launch_add(hipStream_t st, cxd* a, const cxd* b, int64_t n) {
  hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}
void launch_d2f(hipStream_t st, const cxd* a, cxf* b, int64_t n) {
  hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}
void launch_f2d(hipStream_t st, const cxf* a, cxd* b, int64_t n) {
  hipLaunchKernelGGL(k_f2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
}
void launch_norm_partial(hipStream_t st, const cxd* a, int64_t n, int64_t s1, int64_t s2, double* part, int nblk) {
  hipLaunchKernelGGL(k_norm_partial, dim3(nblk), dim3(256), 0, st, a, n, s1, s2, part);
}

}  // namespace vsie
