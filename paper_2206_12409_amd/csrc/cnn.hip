// Learned preconditioner network on the device: forward, backward and Adam for the 3D U-Net of
// cnn.h, with every convolution on the matrix cores (bfloat16 operands, float32 accumulation).
//
// Activations are float32 in HBM, [D][H][W][C] with C padded to a multiple of 16 (padding channels
// hold zeros). A convolution is an implicit GEMM per 3 x 3 x 3 tap: out[v][o] += sum_i in[v + tap][i]
// w[tap][o][i]. A workgroup of four wavefronts owns a 16 (x) by 4 (y) tile of output voxels at one
// z; each wavefront one 16-voxel row, all output channels (up to four 16-wide tiles). Input
// channels are taken 16 at a time: the 3 x 6 x 18 halo of the tile and the chunk's weights of all
// 27 taps are converted to bfloat16 and staged in LDS, then each wavefront runs 27 x (Cout / 16)
// MFMA 16x16x16 steps (A = 16 voxels x 16 input channels, B = 16 input x 16 output channels).
// The decoder inputs [up2(a), b] are read in place (half-resolution reads of a), and the
// backward-data pass multiplies its input gradient by the activation's slope (1 where the layer
// output is positive, LEAK elsewhere) while staging.
//
// Weight gradients: per (output tile, input tile) and z plane, a workgroup accumulates all 27 taps
// over the plane's voxel tiles with MFMA steps whose reduction dimension is the voxels
// (A = output gradient, B = shifted input), reduces its wavefronts in LDS and writes one partial
// per plane; a second kernel sums the planes in a fixed order (deterministic).
#include "cnn.h"

#include <random>

namespace vsie {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f) {
  // round to nearest, ties to even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr float LEAK = 0.1f;   // slope of the activation for negative inputs (leaky ReLU)
__device__ inline float leak_mask(float g, float y) { return y > 0.f ? g : LEAK * g; }

// ---------------------------------------------------------------------------------------------
// convolution forward (also the backward-data pass with reversed, transposed weights)
struct ConvArgs {
  const float* in0;        // channels [0, c0) of the (virtual) input
  const float* in1;        // channels [c0, c0 + c1), full resolution (may be null when c1 = 0)
  const float* mask;       // optional: in0 values multiplied by (mask > 0), same layout as in0
  const uint16_t* w;       // [27][cout_p][cin_p] bfloat16, cin_p = c0 + c1
  const float* bias;       // [cout] or null
  float* out;              // [D][H][W][cout_p]
  int c0, c1, up0, relu, cout_p, cout;
  int D, H, W;
};

constexpr int CT_X = 16, CT_Y = 4;                        // output tile per workgroup
constexpr int HX = CT_X + 2, HY = CT_Y + 2, HV = 3 * HY * HX;   // halo voxels
constexpr int CONV_NT = 4;                                  // output tiles of 16 channels per workgroup

// grid: (x tiles, y tiles, D x output-channel groups of up to 64)
__global__ __launch_bounds__(256) void k_conv3_fwd(ConvArgs a) {
  __shared__ __align__(16) uint16_t tile[HV * 16];
  __shared__ __align__(16) uint16_t wl[27 * CONV_NT * 16 * 16];
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int ngrp = (a.cout_p + 16 * CONV_NT - 1) / (16 * CONV_NT);
  const int x0 = blockIdx.x * CT_X, y0 = blockIdx.y * CT_Y, z = blockIdx.z / ngrp;
  const int grp = blockIdx.z % ngrp;
  const int ob = grp * 16 * CONV_NT;                                  // first output channel
  const int nt = min(CONV_NT, (a.cout_p - ob) / 16);                  // output tiles here
  const int cin_p = a.c0 + a.c1;
  const int Hh = a.H / 2, Wh = a.W / 2;
  f32x4 acc[CONV_NT];
#pragma unroll
  for (int n = 0; n < CONV_NT; ++n) acc[n] = f32x4{0, 0, 0, 0};
  for (int kc = 0; kc < cin_p; kc += 16) {
    __syncthreads();
    // halo of input channels [kc, kc + 16): HV voxels x 4 groups of 4 channels
    for (int e = t; e < HV * 4; e += 256) {
      const int q = e % 4, hv = e / 4;
      const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z + hz - 1;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H && gz >= 0 && gz < a.D) {
        if (kc < a.c0) {
          int64_t vox;
          if (a.up0) vox = ((int64_t)(gz >> 1) * Hh + (gy >> 1)) * Wh + (gx >> 1);
          else vox = ((int64_t)gz * a.H + gy) * a.W + gx;
          v = *reinterpret_cast<const float4*>(a.in0 + vox * a.c0 + kc + 4 * q);
          if (a.mask) {
            const float4 m = *reinterpret_cast<const float4*>(a.mask + vox * a.c0 + kc + 4 * q);
            v.x = leak_mask(v.x, m.x);
            v.y = leak_mask(v.y, m.y);
            v.z = leak_mask(v.z, m.z);
            v.w = leak_mask(v.w, m.w);
          }
        } else {
          const int64_t vox = ((int64_t)gz * a.H + gy) * a.W + gx;
          v = *reinterpret_cast<const float4*>(a.in1 + vox * a.c1 + (kc - a.c0) + 4 * q);
        }
      }
      uint16_t* d = tile + hv * 16 + 4 * q;
      d[0] = to_bf16(v.x);
      d[1] = to_bf16(v.y);
      d[2] = to_bf16(v.z);
      d[3] = to_bf16(v.w);
    }
    // weights of the chunk for this group's output channels: [27][nt * 16][16]
    for (int e = t; e < 27 * nt * 16 * 2; e += 256) {
      const int half = e % 2, o = (e / 2) % (nt * 16), tap = e / (2 * nt * 16);
      const uint4 v = *reinterpret_cast<const uint4*>(a.w + ((int64_t)tap * a.cout_p + ob + o) * cin_p + kc + 8 * half);
      *reinterpret_cast<uint4*>(wl + (tap * CONV_NT * 16 + o) * 16 + 8 * half) = v;
    }
    __syncthreads();
    const int m = lane % 16, g = lane / 16;
#pragma unroll 1
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
      const bf16x4 A = *reinterpret_cast<const bf16x4*>(tile + ((dz * HY + wave + dy) * HX + m + dx) * 16 + 4 * g);
#pragma unroll
      for (int n = 0; n < CONV_NT; ++n)
        if (n < nt) {
          const bf16x4 B = *reinterpret_cast<const bf16x4*>(wl + (tap * CONV_NT * 16 + n * 16 + m) * 16 + 4 * g);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[n], 0, 0, 0);
        }
    }
  }
  // D[m][n]: voxel x0 + 4 (lane / 16) + j, channel ob + n * 16 + lane % 16
  const int y = y0 + wave;
  if (y >= a.H) return;
#pragma unroll
  for (int n = 0; n < CONV_NT; ++n) {
    if (n >= nt) break;
    const int o = ob + n * 16 + lane % 16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + 4 * (lane / 16) + j;
      if (x >= a.W) continue;
      float v = 0.f;
      if (o < a.cout) {
        v = acc[n][j] + (a.bias ? a.bias[o] : 0.f);
        if (a.relu && !(v > 0.f)) v *= LEAK;
      }
      a.out[(((int64_t)z * a.H + y) * a.W + x) * a.cout_p + o] = v;
    }
  }
}

void cnn_conv_forward(hipStream_t st, const float* in0, int c0, bool up0, const float* in1, int c1,
                      const float* mask, const uint16_t* w, const float* bias, bool relu, float* out, int cout_p,
                      int cout, int D, int H, int W) {
  if (c0 % 16 || c1 % 16 || cout_p % 16 || cout_p < 16 || cout > cout_p || c0 < 16 || (c1 > 0 && !in1))
    throw Error(VSIE_E_ARG, "conv: channel counts must be positive multiples of 16");
  if (up0 && (D % 2 || H % 2 || W % 2)) throw Error(VSIE_E_ARG, "conv: upsampled input needs even sizes");
  if (up0 && mask) throw Error(VSIE_E_ARG, "conv: no mask on an upsampled input");
  ConvArgs a{in0, in1, mask, w, bias, out, c0, c1, up0 ? 1 : 0, relu ? 1 : 0, cout_p, cout, D, H, W};
  const int ngrp = (cout_p + 16 * CONV_NT - 1) / (16 * CONV_NT);
  dim3 grid(nblk(W, CT_X), nblk(H, CT_Y), (unsigned)(D * ngrp));
  hipLaunchKernelGGL(k_conv3_fwd, grid, dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------------------------
// weight gradient: gw[o][tap][i] = sum_v g[v][o] in[v + tap][i] (g masked by the ReLU of the
// layer output), gb[o] = sum_v g[v][o]; per (o tile, i tile, z plane) one partial
struct WgradArgs {
  const float* in0;
  const float* in1;
  const float* g;          // [D][H][W][cout_p]
  const float* mask;       // layer output (ReLU mask) or null
  float* part;             // [D][n_ot][n_it][27 * 256 + 16]
  int c0, c1, up0, cout_p;
  int D, H, W;
};

__global__ __launch_bounds__(256) void k_conv3_wgrad(WgradArgs a) {
  __shared__ __align__(16) uint16_t xt[HV * 16];            // input halo, one 16-channel tile
  __shared__ __align__(16) uint16_t gt[CT_Y * CT_X * 16];   // output gradient tile, one 16-channel tile
  __shared__ float red[4][16 * 16];
  const int t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int cin_p = a.c0 + a.c1;
  const int n_it = cin_p / 16, n_ot = a.cout_p / 16;
  const int ot = blockIdx.x / n_it, it = blockIdx.x % n_it;
  const int z = blockIdx.y;
  const int kc = it * 16, oc = ot * 16;
  const int Hh = a.H / 2, Wh = a.W / 2;
  f32x4 acc[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) acc[k] = f32x4{0, 0, 0, 0};
  float bsum = 0.f;
  const int ntx = (a.W + CT_X - 1) / CT_X, nty = (a.H + CT_Y - 1) / CT_Y;
  for (int tt = 0; tt < ntx * nty; ++tt) {
    const int x0 = (tt % ntx) * CT_X, y0 = (tt / ntx) * CT_Y;
    __syncthreads();
    for (int e = t; e < HV * 4; e += 256) {
      const int q = e % 4, hv = e / 4;
      const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z + hz - 1;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H && gz >= 0 && gz < a.D) {
        if (kc < a.c0) {
          int64_t vox;
          if (a.up0) vox = ((int64_t)(gz >> 1) * Hh + (gy >> 1)) * Wh + (gx >> 1);
          else vox = ((int64_t)gz * a.H + gy) * a.W + gx;
          v = *reinterpret_cast<const float4*>(a.in0 + vox * a.c0 + kc + 4 * q);
        } else {
          const int64_t vox = ((int64_t)gz * a.H + gy) * a.W + gx;
          v = *reinterpret_cast<const float4*>(a.in1 + vox * a.c1 + (kc - a.c0) + 4 * q);
        }
      }
      uint16_t* d = xt + hv * 16 + 4 * q;
      d[0] = to_bf16(v.x);
      d[1] = to_bf16(v.y);
      d[2] = to_bf16(v.z);
      d[3] = to_bf16(v.w);
    }
    for (int e = t; e < CT_Y * CT_X * 4; e += 256) {
      const int q = e % 4, v = e / 4;
      const int x = x0 + v % CT_X, y = y0 + v / CT_X;
      float4 gv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (x < a.W && y < a.H) {
        const int64_t vox = ((int64_t)z * a.H + y) * a.W + x;
        gv = *reinterpret_cast<const float4*>(a.g + vox * a.cout_p + oc + 4 * q);
        if (a.mask) {
          const float4 m = *reinterpret_cast<const float4*>(a.mask + vox * a.cout_p + oc + 4 * q);
          gv.x = leak_mask(gv.x, m.x);
          gv.y = leak_mask(gv.y, m.y);
          gv.z = leak_mask(gv.z, m.z);
          gv.w = leak_mask(gv.w, m.w);
        }
      }
      uint16_t* d = gt + v * 16 + 4 * q;
      d[0] = to_bf16(gv.x);
      d[1] = to_bf16(gv.y);
      d[2] = to_bf16(gv.z);
      d[3] = to_bf16(gv.w);
    }
    __syncthreads();
    // this wavefront's 16 voxels: the row y0 + wave; A[o][k = voxel] and B[k = voxel][i]
    const int m = lane % 16, g = lane / 16;
    bf16x4 A;
#pragma unroll
    for (int j = 0; j < 4; ++j) A[j] = (short)gt[(wave * CT_X + 4 * g + j) * 16 + m];
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
      bf16x4 B;
#pragma unroll
      for (int j = 0; j < 4; ++j) B[j] = (short)xt[((dz * HY + wave + dy) * HX + 4 * g + j + dx) * 16 + m];
      acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[tap], 0, 0, 0);
    }
    // bias: float32 sum of the masked gradient over the tile (first input tile only)
    if (it == 0 && t < 16 * CT_Y) {
      const int o = t % 16, yy = y0 + t / 16;
      if (yy < a.H)
        for (int xx = x0; xx < min(x0 + CT_X, a.W); ++xx) {
          const int64_t vox = ((int64_t)z * a.H + yy) * a.W + xx;
          float gv = a.g[vox * a.cout_p + oc + o];
          if (a.mask) gv = leak_mask(gv, a.mask[vox * a.cout_p + oc + o]);
          bsum += gv;
        }
    }
  }
  // reduce the four wavefronts tap by tap; D[m = o][n = i]: o = 4 (lane / 16) + j, i = lane % 16
  float* out = a.part + (((int64_t)z * n_ot + ot) * n_it + it) * (27 * 256 + 16);
  for (int tap = 0; tap < 27; ++tap) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][(4 * (lane / 16) + j) * 16 + lane % 16] = acc[tap][j];
    __syncthreads();
    out[tap * 256 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
  }
  if (it == 0) {
    __syncthreads();
    red[0][t] = bsum;   // t < 64: (o = t % 16, row t / 16)
    __syncthreads();
    if (t < 16) out[27 * 256 + t] = (red[0][t] + red[0][16 + t]) + (red[0][32 + t] + red[0][48 + t]);
  }
}

// sum the plane partials in order: gw[o][tap][i] (o < cout, i < cin), gb[o]
__global__ void k_wgrad_reduce(const float* __restrict__ part, int D, int n_ot, int n_it, int cout, int cin,
                               int c0, int cin0, float* __restrict__ gw, float* __restrict__ gb) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)cout * 27 * cin;
  if (e < nw) {
    const int i = (int)(e % cin), tap = (int)((e / cin) % 27), o = (int)(e / (27LL * cin));
    // storage channel of real input channel i: the first input keeps its padded width c0
    const int is = i < cin0 ? i : c0 + (i - cin0);
    const int ot = o / 16, it = is / 16;
    float s = 0.f;
    for (int z = 0; z < D; ++z)
      s += part[(((int64_t)z * n_ot + ot) * n_it + it) * (27 * 256 + 16) + tap * 256 + (o % 16) * 16 + is % 16];
    gw[e] = s;
  } else if (e < nw + cout) {
    const int o = (int)(e - nw);
    float s = 0.f;
    for (int z = 0; z < D; ++z) s += part[(((int64_t)z * n_ot + o / 16) * n_it + 0) * (27 * 256 + 16) + 27 * 256 + o % 16];
    gb[o] = s;
  }
}

// ---------------------------------------------------------------------------------------------
// elementwise pieces
__global__ void k_pool2(const float* __restrict__ in, float* __restrict__ out, int D, int H, int W, int C) {
  const int Dh = D / 2, Hh = H / 2, Wh = W / 2;
  const int64_t n = (int64_t)Dh * Hh * Wh * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t v = e / C;
    const int x = (int)(v % Wh), y = (int)((v / Wh) % Hh), z = (int)(v / ((int64_t)Wh * Hh));
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          s += in[(((int64_t)(2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx) * C + c];
    out[e] = 0.125f * s;
  }
}

// g_full += up2(g_half) / 8 (gradient of avgpool2), full-resolution sizes D, H, W
__global__ void k_pool2_bwd_add(const float* __restrict__ gh, float* __restrict__ gf, int D, int H, int W, int C) {
  const int64_t n = (int64_t)D * H * W * C;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int64_t v = e / C;
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((int64_t)W * H));
    gf[e] += 0.125f * gh[((((int64_t)(z >> 1) * (H / 2)) + (y >> 1)) * (W / 2) + (x >> 1)) * C + c];
  }
}

// gradient of a decoder input [up2(a), b]: ga (half resolution, ca channels) = 2x2x2 sums of the
// first ca channels of gcat, gb (full resolution, cb channels) = the rest; both overwritten
__global__ void k_cat_bwd(const float* __restrict__ gcat, int D, int H, int W, int ca, int cb, float* __restrict__ ga,
                          float* __restrict__ gb) {
  const int C = ca + cb;
  const int64_t nb = (int64_t)D * H * W * cb, na = (int64_t)(D / 2) * (H / 2) * (W / 2) * ca;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nb + na; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nb) {
      const int c = (int)(e % cb);
      gb[e] = gcat[(e / cb) * C + ca + c];
    } else {
      const int64_t f = e - nb;
      const int c = (int)(f % ca);
      const int64_t v = f / ca;
      const int Wh = W / 2, Hh = H / 2;
      const int x = (int)(v % Wh), y = (int)((v / Wh) % Hh), z = (int)(v / ((int64_t)Wh * Hh));
      float s = 0.f;
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx)
            s += gcat[(((int64_t)(2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx) * C + c];
      ga[f] = s;
    }
  }
}

// g = (y - t) / n on the first nreal channels (zero elsewhere); per-block partial sums of (y - t)^2
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ tg, int64_t nvox, int C, int nreal,
                            float* __restrict__ g, double* __restrict__ part) {
  __shared__ double sh[256];
  const double inv_n = 1.0 / ((double)nvox * nreal);
  double s = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvox * C; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    float d = 0.f;
    if (c < nreal) {
      d = y[e] - tg[e];
      s += (double)d * d;
    }
    g[e] = (float)(d * inv_n);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_parts_d(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = scale * s;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 GEMM layouts of one layer: wf[tap][o][i] = w[o][tap][i], wb[tap][i][o] = w[o][26 - tap][i]
// (storage channels; input channel i of the real layout maps to storage channel is)
__global__ void k_pack_weights(const float* __restrict__ w, int cout, int cin, int cin0, int c0, int cout_p,
                               int cin_p, uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
  const int64_t n = 27LL * cout_p * cin_p;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int is = (int)(e % cin_p), o = (int)((e / cin_p) % cout_p), tap = (int)(e / ((int64_t)cin_p * cout_p));
  // real input channel of storage channel is: the first input occupies [0, c0) with cin0 real
  int i = -1;
  if (is < c0) i = is < cin0 ? is : -1;
  else i = cin0 + (is - c0);
  float v = 0.f, vb = 0.f;
  if (o < cout && i >= 0 && i < cin) {
    v = w[((int64_t)o * 27 + tap) * cin + i];
    vb = w[((int64_t)o * 27 + (26 - tap)) * cin + i];
  }
  wf[((int64_t)tap * cout_p + o) * cin_p + is] = to_bf16(v);
  wb[((int64_t)tap * cin_p + is) * cout_p + o] = to_bf16(vb);
}

// ---------------------------------------------------------------------------------------------
// host side
static const struct {
  int cin, cout, cin0, c0;   // real channels; real and storage channels of the first input part
  bool relu;
} kLayers[CNN_NLAYER] = {
    {CNN_IN, 16, CNN_IN, 16, true}, {16, 16, 16, 16, true},  {16, 32, 16, 16, true}, {32, 32, 32, 32, true},
    {32, 48, 32, 32, true},         {48, 48, 48, 48, true},  {48, 64, 48, 48, true}, {64, 64, 64, 64, true},
    {112, 48, 64, 64, true},        {80, 32, 48, 48, true},  {48, 16, 32, 32, true}, {16, CNN_OUT, 16, 16, false},
};
static int pad16(int c) { return (c + 15) / 16 * 16; }

Cnn::~Cnn() {
  for (void* p : owned) (void)hipFree(p);
}

template <typename T> static T* cnn_alloc(Cnn& N, int64_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess)
    throw Error(VSIE_E_NOMEM, "hipMalloc for the network failed");
  N.owned.push_back(p);
  VSIE_HIP(hipMemset(p, 0, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
  return (T*)p;
}

void cnn_init(Cnn& N, uint64_t seed) {
  int64_t off = 0, wf = 0, wb = 0;
  for (int l = 0; l < CNN_NLAYER; ++l) {
    CnnLayerDesc& d = N.L[l];
    d.cin = kLayers[l].cin;
    d.cout = kLayers[l].cout;
    d.relu = kLayers[l].relu;
    d.cout_p = pad16(d.cout);
    d.cin_p = kLayers[l].c0 + pad16(d.cin - kLayers[l].cin0);
    d.w_off = off;
    off += (int64_t)d.cout * 27 * d.cin;
    d.b_off = off;
    off += d.cout;
    d.wf_off = wf;
    wf += 27LL * d.cout_p * d.cin_p;
    d.wb_off = wb;
    wb += 27LL * d.cout_p * d.cin_p;
  }
  N.nparam = off;
  N.nwf = wf;
  N.nwb = wb;
  N.params = cnn_alloc<float>(N, off);
  N.grads = cnn_alloc<float>(N, off);
  N.adam_m = cnn_alloc<float>(N, off);
  N.adam_v = cnn_alloc<float>(N, off);
  N.wf = cnn_alloc<uint16_t>(N, wf);
  N.wb = cnn_alloc<uint16_t>(N, wb);
  N.red = cnn_alloc<double>(N, 4096);
  std::vector<float> h((size_t)off, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 0; l < CNN_NLAYER; ++l) {
    const CnnLayerDesc& d = N.L[l];
    const double sd = std::sqrt(2.0 / (27.0 * d.cin));
    for (int64_t i = 0; i < (int64_t)d.cout * 27 * d.cin; ++i) h[d.w_off + i] = (float)(sd * nd(rng));
  }
  VSIE_HIP(hipMemcpy(N.params, h.data(), sizeof(float) * off, hipMemcpyHostToDevice));
  N.step = 0;
}

void cnn_refresh_weights(Cnn& N, hipStream_t st) {
  for (int l = 0; l < CNN_NLAYER; ++l) {
    const CnnLayerDesc& d = N.L[l];
    const int64_t n = 27LL * d.cout_p * d.cin_p;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(n, 256)), dim3(256), 0, st, N.params + d.w_off, d.cout, d.cin,
                       kLayers[l].cin0, kLayers[l].c0, d.cout_p, d.cin_p, N.wf + d.wf_off, N.wb + d.wb_off);
  }
  VSIE_HIP(hipGetLastError());
}

// level (resolution) of each layer and the buffers it reads
static int layer_level(int l) {
  static const int lv[CNN_NLAYER] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 1, 0, 0};
  return lv[l];
}

void cnn_size(Cnn& N, int D, int H, int W) {
  if (D % 8 || H % 8 || W % 8 || D <= 0 || H <= 0 || W <= 0)
    throw Error(VSIE_E_ARG, "network grid sizes must be positive multiples of 8");
  if (N.D == D && N.H == H && N.W == W) return;
  for (void* p : N.bufs) (void)hipFree(p);
  N.bufs.clear();
  N.D = D;
  N.H = H;
  N.W = W;
  auto alloc = [&](int64_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(float) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess)
      throw Error(VSIE_E_NOMEM, "hipMalloc for the network activations failed");
    VSIE_HIP(hipMemset(p, 0, sizeof(float) * (size_t)std::max<int64_t>(n, 1)));
    N.bufs.push_back(p);
    return (float*)p;
  };
  const int64_t V0 = (int64_t)D * H * W;
  auto vox = [&](int lv) { return V0 >> (3 * lv); };
  for (int l = 0; l < CNN_NLAYER; ++l) {
    N.act[l] = alloc(vox(layer_level(l)) * N.L[l].cout_p);
    N.gact[l] = alloc(vox(layer_level(l)) * N.L[l].cout_p);
  }
  const int pc[3] = {16, 32, 48};
  for (int k = 0; k < 3; ++k) {
    N.pool[k] = alloc(vox(k + 1) * pc[k]);
    N.gpool[k] = alloc(vox(k + 1) * pc[k]);
  }
  N.gcat = alloc(std::max({vox(0) * N.L[10].cin_p, vox(1) * N.L[9].cin_p, vox(2) * N.L[8].cin_p}));
  N.x_in = alloc(V0 * 16);
  N.target = alloc(V0 * 16);
  int64_t wp = 0;
  for (int l = 0; l < CNN_NLAYER; ++l) {
    const int lv = layer_level(l);
    wp = std::max<int64_t>(wp, (int64_t)(D >> lv) * (N.L[l].cout_p / 16) * (N.L[l].cin_p / 16) * (27 * 256 + 16));
  }
  N.wpart = alloc(wp);
  N.wpart_elems = wp;
}

// input buffers of layer l: (in0, c0, up0, in1, c1)
struct LayerIn {
  const float* in0;
  int c0;
  bool up0;
  const float* in1;
  int c1;
};
static LayerIn layer_inputs(const Cnn& N, int l) {
  switch (l) {
    case 0: return {N.x_in, 16, false, nullptr, 0};
    case 1: return {N.act[0], 16, false, nullptr, 0};
    case 2: return {N.pool[0], 16, false, nullptr, 0};
    case 3: return {N.act[2], 32, false, nullptr, 0};
    case 4: return {N.pool[1], 32, false, nullptr, 0};
    case 5: return {N.act[4], 48, false, nullptr, 0};
    case 6: return {N.pool[2], 48, false, nullptr, 0};
    case 7: return {N.act[6], 64, false, nullptr, 0};
    case 8: return {N.act[7], 64, true, N.act[5], 48};
    case 9: return {N.act[8], 48, true, N.act[3], 32};
    case 10: return {N.act[9], 32, true, N.act[1], 16};
    default: return {N.act[10], 16, false, nullptr, 0};
  }
}

void cnn_forward(Cnn& N, hipStream_t st) {
  for (int l = 0; l < CNN_NLAYER; ++l) {
    const int lv = layer_level(l);
    const int D = N.D >> lv, H = N.H >> lv, W = N.W >> lv;
    if (l == 2 || l == 4 || l == 6) {   // pool the level above first
      const int k = l / 2 - 1;
      const int src = l - 1;
      const int C = N.L[src].cout_p;
      const int64_t n = (int64_t)D * H * W * C;
      hipLaunchKernelGGL(k_pool2, dim3(std::min<unsigned>(nblk(n, 256), 16384)), dim3(256), 0, st, N.act[src],
                         N.pool[k], 2 * D, 2 * H, 2 * W, C);
    }
    const CnnLayerDesc& d = N.L[l];
    const LayerIn in = layer_inputs(N, l);
    cnn_conv_forward(st, in.in0, in.c0, in.up0, in.in1, in.c1, nullptr, N.wf + d.wf_off, N.params + d.b_off, d.relu,
                     N.act[l], d.cout_p, d.cout, D, H, W);
  }
  VSIE_HIP(hipGetLastError());
}

void cnn_conv_wgrad(Cnn& N, hipStream_t st, int layer, const float* in0, int c0, bool up0, const float* in1, int c1,
                    const float* g, const float* mask, int cout_p, float* gw, float* gb, int D, int H, int W) {
  const CnnLayerDesc& d = N.L[layer];
  const int n_ot = cout_p / 16, n_it = (c0 + c1) / 16;
  if (c0 % 16 || c1 % 16 || cout_p % 16 || c0 + c1 != d.cin_p || cout_p != d.cout_p || (c1 > 0 && !in1))
    throw Error(VSIE_E_ARG, "wgrad: channel counts do not match the layer");
  if (up0 && (D % 2 || H % 2 || W % 2)) throw Error(VSIE_E_ARG, "wgrad: upsampled input needs even sizes");
  const int64_t need = (int64_t)D * n_ot * n_it * (27 * 256 + 16);
  if (need > N.wpart_elems) {   // a layer on a grid the network was not sized for (tests)
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(float) * (size_t)need) != hipSuccess) throw Error(VSIE_E_NOMEM, "wgrad partials");
    N.owned.push_back(p);
    N.wpart = (float*)p;
    N.wpart_elems = need;
  }
  WgradArgs a{in0, in1, g, mask, N.wpart, c0, c1, up0 ? 1 : 0, cout_p, D, H, W};
  hipLaunchKernelGGL(k_conv3_wgrad, dim3((unsigned)(n_ot * n_it), (unsigned)D), dim3(256), 0, st, a);
  const int64_t n = (int64_t)d.cout * 27 * d.cin + d.cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk(n, 256)), dim3(256), 0, st, N.wpart, D, n_ot, n_it, d.cout, d.cin,
                     kLayers[layer].c0, kLayers[layer].cin0, gw, gb);
}

void cnn_backward(Cnn& N, hipStream_t st) {
  const int64_t V0 = (int64_t)N.D * N.H * N.W;
  // loss and its gradient
  const unsigned nb = std::min<unsigned>(nblk(V0 * 16, 256), 2048);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, st, N.act[11], N.target, V0, 16, CNN_OUT, N.gact[11],
                     N.red + 8);
  hipLaunchKernelGGL(k_sum_parts_d, dim3(1), dim3(64), 0, st, N.red + 8, (int)nb, 0.5 / ((double)V0 * CNN_OUT), N.red);
  for (int l = CNN_NLAYER - 1; l >= 0; --l) {
    const int lv = layer_level(l);
    const int D = N.D >> lv, H = N.H >> lv, W = N.W >> lv;
    const CnnLayerDesc& d = N.L[l];
    const LayerIn in = layer_inputs(N, l);
    const float* mask = d.relu ? N.act[l] : nullptr;
    cnn_conv_wgrad(N, st, l, in.in0, in.c0, in.up0, in.in1, in.c1, N.gact[l], mask, d.cout_p, N.grads + d.w_off,
                   N.grads + d.b_off, D, H, W);
    if (l == 0) break;
    // gradient with respect to the layer input: forward convolution of the masked output gradient
    // with the reversed, transposed weights
    float* gin;
    int gin_c = d.cin_p;
    if (l >= 8 && l <= 10) gin = N.gcat;
    else if (l == 2 || l == 4 || l == 6) gin = N.gpool[l / 2 - 1];
    else gin = N.gact[l - 1];
    cnn_conv_forward(st, N.gact[l], d.cout_p, false, nullptr, 0, mask, N.wb + d.wb_off, nullptr, false, gin, gin_c,
                     gin_c, D, H, W);
    if (l >= 8 && l <= 10) {
      // [up2(a), b]: a = act[prev decoder or e4], b = the skip
      const int ca = in.c0, cb = in.c1;
      float* ga = l == 8 ? N.gact[7] : N.gact[l - 1];
      float* gbuf = l == 8 ? N.gact[5] : (l == 9 ? N.gact[3] : N.gact[1]);
      const int64_t n = (int64_t)D * H * W * cb + (int64_t)(D / 2) * (H / 2) * (W / 2) * ca;
      hipLaunchKernelGGL(k_cat_bwd, dim3(std::min<unsigned>(nblk(n, 256), 16384)), dim3(256), 0, st, N.gcat, D, H, W, ca,
                         cb, ga, gbuf);
    } else if (l == 2 || l == 4 || l == 6) {
      // the pooled input: add its gradient to that of the level above's output (act[l - 1])
      const int C = N.L[l - 1].cout_p;
      const int64_t n = (int64_t)(2 * D) * (2 * H) * (2 * W) * C;
      hipLaunchKernelGGL(k_pool2_bwd_add, dim3(std::min<unsigned>(nblk(n, 256), 16384)), dim3(256), 0, st,
                         N.gpool[l / 2 - 1], N.gact[l - 1], 2 * D, 2 * H, 2 * W, C);
    }
  }
  VSIE_HIP(hipGetLastError());
}

void cnn_adam(Cnn& N, float lr, hipStream_t st) {
  N.step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - (float)std::pow(0.9, (double)N.step), c2 = 1.f - (float)std::pow(0.999, (double)N.step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(N.nparam, 256)), dim3(256), 0, st, N.params, N.grads, N.adam_m, N.adam_v,
                     N.nparam, lr, b1, b2, c1, c2, 1e-8f);
  cnn_refresh_weights(N, st);
}

}  // namespace vsie
