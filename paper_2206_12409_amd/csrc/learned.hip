// Learned preconditioner of the reduced (far-eliminated) system: the network of cnn.hip on the
// body currents, its training pairs, its training loop and its application inside flexible GMRES.
//
// The base right preconditioner M is block diagonal (inverse reduced near block, inverse body
// diagonal D^-1). The learned one adds a body correction: P(v) = M v + s c N(v_b / s, m), with
// s the RMS of the body part v_b, m = D^-1 / c the material channels and c the largest |D^-1| of
// the tissue. Training pairs come from the plain preconditioned GMRES solves: each Arnoldi step
// applies the reduced operator A_S to z = M v, so w = A_S z has the exact correction z; the pair
// is (input w_b / s, target (z_b - D^-1 w_b) / (s c)) with s the RMS of w_b, i.e. the network
// learns what M misses of A_S^-1 on the body.
#include <algorithm>
#include <random>

#include "cnn.h"
#include "kernels.h"

namespace vsie {

static unsigned nb256(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65535); }

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// per-block partial sums of |v|^2 over the 3 nv body entries, then the RMS over the tissue
// entries (3 n_tissue) into *scale (0 when the body part vanishes)
__global__ void k_body_sumsq(const cxd* __restrict__ vb, int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += vb[i].re * vb[i].re + vb[i].im * vb[i].im;
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_rms(const double* __restrict__ part, int np, double count, double* __restrict__ scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < np; ++i) s += part[i];
    *scale = count > 0 ? sqrt(s / count) : 0.0;
  }
}

// network input [D][H][W][16] from a body vector (three components of nv values each, voxel
// (i1, i2, i3) at i1 + n1 (i2 + n2 i3)) scaled by 1 / *scale, and the material channels
__global__ void k_net_input(const cxd* __restrict__ vb, const float2* __restrict__ mat, const double* __restrict__ scale,
                            int n1, int n2, int n3, int D, int H, int W, float* __restrict__ x) {
  const int64_t nvox = (int64_t)D * H * W;
  const double s = *scale;
  const double inv = s > 0 ? 1.0 / s : 0.0;
  const int64_t nv = (int64_t)n1 * n2 * n3;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvox; e += (int64_t)gridDim.x * blockDim.x) {
    const int xx = (int)(e % W), yy = (int)((e / W) % H), zz = (int)(e / ((int64_t)W * H));
    float* o = x + e * 16;
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (xx < n1 && yy < n2 && zz < n3) {
      const int64_t p = xx + (int64_t)n1 * (yy + (int64_t)n2 * zz);
      const float2 m = mat[p];
      if (m.x != 0.f || m.y != 0.f) {   // tissue voxel
        for (int c = 0; c < 3; ++c) {
          const cxd a = vb[c * nv + p];
          v[2 * c] = (float)(a.re * inv);
          v[2 * c + 1] = (float)(a.im * inv);
        }
        v[6] = m.x;
        v[7] = m.y;
      }
    }
    for (int c = 0; c < 8; ++c) o[c] = v[c];
    for (int c = 8; c < 16; ++c) o[c] = 0.f;
  }
}

// out_b += (*scale) c y on the tissue voxels (y = network output, channels Re/Im of x, y, z)
__global__ void k_net_output_add(const float* __restrict__ y, const float2* __restrict__ mat,
                                 const double* __restrict__ scale, double c, int n1, int n2, int n3, int H, int W,
                                 cxd* __restrict__ ob) {
  const int64_t nv = (int64_t)n1 * n2 * n3;
  const double s = *scale * c;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nv; p += (int64_t)gridDim.x * blockDim.x) {
    const float2 m = mat[p];
    if (m.x == 0.f && m.y == 0.f) continue;
    const int xx = (int)(p % n1), yy = (int)((p / n1) % n2), zz = (int)(p / ((int64_t)n1 * n2));
    const float* yv = y + (((int64_t)zz * H + yy) * W + xx) * 16;
    for (int comp = 0; comp < 3; ++comp) {
      cxd& o = ob[comp * nv + p];
      o.re += s * yv[2 * comp];
      o.im += s * yv[2 * comp + 1];
    }
  }
}

// training pair p: [D][H][W][16] bfloat16, channels 0..7 input, 8..13 target
// A pair whose body part carries less than PAIR_MIN_BODY of the coupled vector's norm is stored
// as zeros (it teaches nothing the body network can see: its correction comes from the near
// currents, e.g. the product of a restart, whose body part is only the residual).
constexpr double PAIR_MIN_BODY = 0.3;

__global__ void k_pack_pair(const cxd* __restrict__ wb, const cxd* __restrict__ zb, const cxd* __restrict__ dw,
                            const float2* __restrict__ mat, const double* __restrict__ scale,
                            const double* __restrict__ wnorm, double nbody, double c, int n1, int n2, int n3, int D,
                            int H, int W, uint16_t* __restrict__ pair) {
  const int64_t nvox = (int64_t)D * H * W, nv = (int64_t)n1 * n2 * n3;
  const double s = *scale;
  const bool keep = s > 0 && s * sqrt(nbody) >= PAIR_MIN_BODY * *wnorm;
  const double inv = keep ? 1.0 / s : 0.0, invt = keep ? 1.0 / (s * c) : 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvox; e += (int64_t)gridDim.x * blockDim.x) {
    const int xx = (int)(e % W), yy = (int)((e / W) % H), zz = (int)(e / ((int64_t)W * H));
    float v[16];
    for (int k = 0; k < 16; ++k) v[k] = 0.f;
    if (xx < n1 && yy < n2 && zz < n3) {
      const int64_t p = xx + (int64_t)n1 * (yy + (int64_t)n2 * zz);
      const float2 m = mat[p];
      if (keep && (m.x != 0.f || m.y != 0.f)) {
        for (int comp = 0; comp < 3; ++comp) {
          const cxd a = wb[comp * nv + p];
          v[2 * comp] = (float)(a.re * inv);
          v[2 * comp + 1] = (float)(a.im * inv);
          const cxd zt = zb[comp * nv + p], d = dw[comp * nv + p];
          v[8 + 2 * comp] = (float)((zt.re - d.re) * invt);
          v[8 + 2 * comp + 1] = (float)((zt.im - d.im) * invt);
        }
        v[6] = m.x;
        v[7] = m.y;
      }
    }
    uint16_t* o = pair + e * 16;
    for (int k = 0; k < 16; ++k) o[k] = f2bf(v[k]);
  }
}

// network input and target of a stored pair, both multiplied by exp(i theta) (the map the
// network learns is complex linear, so a common phase is an exact symmetry of the data)
__global__ void k_load_pair(const uint16_t* __restrict__ pair, int64_t nvox, float cth, float sth, float* __restrict__ x,
                            float* __restrict__ t) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvox; e += (int64_t)gridDim.x * blockDim.x) {
    const uint16_t* p = pair + e * 16;
    float* xo = x + e * 16;
    float* to = t + e * 16;
    for (int comp = 0; comp < 3; ++comp) {
      const float re = bf2f(p[2 * comp]), im = bf2f(p[2 * comp + 1]);
      xo[2 * comp] = cth * re - sth * im;
      xo[2 * comp + 1] = sth * re + cth * im;
      const float tr = bf2f(p[8 + 2 * comp]), ti = bf2f(p[8 + 2 * comp + 1]);
      to[2 * comp] = cth * tr - sth * ti;
      to[2 * comp + 1] = sth * tr + cth * ti;
    }
    xo[6] = bf2f(p[6]);
    xo[7] = bf2f(p[7]);
    for (int c = 8; c < 16; ++c) xo[c] = 0.f;
    for (int c = 6; c < 16; ++c) to[c] = 0.f;
  }
}

__global__ void k_accum_d(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

static int round8(int n) { return (n + 7) / 8 * 8; }

void build_material(Handle& H, const std::vector<cxd>& inv) {
  // D^-1 of component 0 (the three are equal) over the tissue, scaled by its largest modulus
  double dmax = 0;
  for (int p = 0; p < H.nv; ++p)
    if (H.chi[p].re != 0 || H.chi[p].im != 0) dmax = std::max(dmax, std::hypot(inv[p].re, inv[p].im));
  std::vector<float> m(2 * (size_t)H.nv, 0.f);
  if (dmax > 0)
    for (int p = 0; p < H.nv; ++p)
      if (H.chi[p].re != 0 || H.chi[p].im != 0) {
        m[2 * (size_t)p] = (float)(inv[p].re / dmax);
        m[2 * (size_t)p + 1] = (float)(inv[p].im / dmax);
        if (m[2 * (size_t)p] == 0.f && m[2 * (size_t)p + 1] == 0.f) m[2 * (size_t)p] = 1e-30f;   // keep the tissue flag
      }
  if (!H.d_material) H.d_material = H.dalloc<float>(2LL * H.nv);
  VSIE_HIP(hipMemcpy(H.d_material, m.data(), sizeof(float) * m.size(), hipMemcpyHostToDevice));
  H.mat_scale = dmax;
}

static void net_grid(const Handle& H, int& D, int& Hh, int& W) {
  D = round8(H.n[2]);
  Hh = round8(H.n[1]);
  W = round8(H.n[0]);
}

// out_full (body rows) += learned correction of v_full's body part
void net_apply(Handle& H, NetState& S, const cxd* v_full, cxd* out_full, hipStream_t st) {
  int D, Hg, W;
  net_grid(H, D, Hg, W);
  cnn_size(S.N, D, Hg, W);
  const int64_t off = H.mf + H.mn, nb = 3LL * H.nv;
  const unsigned blocks = 256;
  hipLaunchKernelGGL(k_body_sumsq, dim3(blocks), dim3(256), 0, st, v_full + off, nb, S.N.red + 2560);
  hipLaunchKernelGGL(k_rms, dim3(1), dim3(64), 0, st, S.N.red + 2560, (int)blocks, 3.0 * H.tissue.size(), S.N.red + 1);
  hipLaunchKernelGGL(k_net_input, dim3(nb256((int64_t)D * Hg * W)), dim3(256), 0, st, v_full + off,
                     (const float2*)H.d_material, S.N.red + 1, H.n[0], H.n[1], H.n[2], D, Hg, W, S.N.x_in);
  cnn_forward(S.N, st);
  hipLaunchKernelGGL(k_net_output_add, dim3(nb256(H.nv)), dim3(256), 0, st, S.N.act[CNN_NLAYER - 1],
                     (const float2*)H.d_material, S.N.red + 1, H.mat_scale, H.n[0], H.n[1], H.n[2], Hg, W,
                     out_full + off);
  VSIE_HIP(hipGetLastError());
}

// store the pair (A_S z, z) of one Arnoldi step; dw_tmp: 3 nv scratch for D^-1 w_b
void net_collect_pair(Handle& H, NetState& S, const cxd* z_full, const cxd* w_full, cxd* dw_tmp, hipStream_t st) {
  if (S.count >= S.cap) return;
  int D, Hg, W;
  net_grid(H, D, Hg, W);
  if (S.count == 0 && S.pairs == nullptr) {
    S.D = D;
    S.H = Hg;
    S.W = W;
    const size_t bytes = sizeof(uint16_t) * 16 * (size_t)D * Hg * W * (size_t)S.cap;
    if (hipMalloc(&S.pairs, bytes) != hipSuccess) {
      S.pairs = nullptr;
      throw Error(VSIE_E_NOMEM, "hipMalloc of the training pairs failed");
    }
  }
  if (S.D != D || S.H != Hg || S.W != W) throw Error(VSIE_E_ARG, "training pairs of one network share one grid");
  const int64_t off = H.mf + H.mn, nb = 3LL * H.nv;
  const unsigned blocks = 256;
  launch_mul_diag<double>(st, w_full + off, H.schur.d64.invdiag, dw_tmp, nb);
  hipLaunchKernelGGL(k_body_sumsq, dim3(blocks), dim3(256), 0, st, w_full + off, nb, S.N.red + 2560);
  hipLaunchKernelGGL(k_rms, dim3(1), dim3(64), 0, st, S.N.red + 2560, (int)blocks, 3.0 * H.tissue.size(), S.N.red + 2);
  // norm of the coupled part of w (near currents and body)
  hipLaunchKernelGGL(k_body_sumsq, dim3(blocks), dim3(256), 0, st, w_full + H.mf, (int64_t)H.mn + nb, S.N.red + 2560);
  hipLaunchKernelGGL(k_rms, dim3(1), dim3(64), 0, st, S.N.red + 2560, (int)blocks, 1.0, S.N.red + 4);
  uint16_t* dst = S.pairs + (size_t)S.count * 16 * D * Hg * W;
  hipLaunchKernelGGL(k_pack_pair, dim3(nb256((int64_t)D * Hg * W)), dim3(256), 0, st, w_full + off, z_full + off,
                     dw_tmp, (const float2*)H.d_material, S.N.red + 2, S.N.red + 4, 3.0 * H.tissue.size(),
                     H.mat_scale, H.n[0], H.n[1], H.n[2], D, Hg, W, dst);
  VSIE_HIP(hipGetLastError());
  S.count += 1;
}

NetState::~NetState() {
  if (pairs) (void)hipFree(pairs);
}

double net_train(NetState& S, int epochs, float lr, uint64_t seed, hipStream_t st) {
  if (S.count == 0) throw Error(VSIE_E_STATE, "no training pairs collected");
  cnn_size(S.N, S.D, S.H, S.W);
  cnn_refresh_weights(S.N, st);
  const int64_t nvox = (int64_t)S.D * S.H * S.W;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> ang(0.0, 2.0 * PI);
  std::vector<int> order(S.count);
  double last = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int i = 0; i < (int)S.count; ++i) order[i] = i;
    std::shuffle(order.begin(), order.end(), rng);
    VSIE_HIP(hipMemsetAsync(S.N.red + 3, 0, sizeof(double), st));
    for (int i = 0; i < (int)S.count; ++i) {
      const double th = ang(rng);
      hipLaunchKernelGGL(k_load_pair, dim3(nb256(nvox)), dim3(256), 0, st, S.pairs + (size_t)order[i] * 16 * nvox, nvox,
                         (float)cos(th), (float)sin(th), S.N.x_in, S.N.target);
      cnn_forward(S.N, st);
      cnn_backward(S.N, st);
      hipLaunchKernelGGL(k_accum_d, dim3(1), dim3(64), 0, st, S.N.red, S.N.red + 3);
      cnn_adam(S.N, lr, st);
    }
    double sum = 0;
    VSIE_HIP(hipMemcpyAsync(&sum, S.N.red + 3, sizeof(double), hipMemcpyDeviceToHost, st));
    VSIE_HIP(hipStreamSynchronize(st));
    last = sum / (double)S.count;
  }
  return last;
}

}  // namespace vsie
