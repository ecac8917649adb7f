// Learned preconditioner: a 3D convolutional U-Net on the voxel grid, trained and applied on the
// device with bfloat16 matrix-core convolutions and float32 accumulation (cnn.hip).
#pragma once
#include "vsie_internal.h"

namespace vsie {

constexpr int CNN_NLAYER = 12;
constexpr int CNN_IN = 8;      // six residual channels (Re, Im of x, y, z) and two material channels
constexpr int CNN_OUT = 6;     // correction of the body currents (Re, Im of x, y, z)

struct CnnLayerDesc {
  int cin, cout;        // real channels
  int cin_p, cout_p;    // storage channels (multiples of 16)
  bool relu;
  int64_t w_off, b_off; // offsets into the flat float32 parameter vector (w: [cout][27][cin])
  int64_t wf_off;       // bf16 forward weights [27][cout_p][cin_p]
  int64_t wb_off;       // bf16 backward-data weights [27][cin_p][cout_p] (taps reversed)
};

// The network, its optimiser state, and (when sized for a grid) its activations.
struct Cnn {
  CnnLayerDesc L[CNN_NLAYER];
  int64_t nparam = 0, nwf = 0, nwb = 0;
  float* params = nullptr;       // float32 master parameters
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wf = nullptr;        // bf16 weights in the GEMM layouts
  uint16_t* wb = nullptr;
  int64_t step = 0;              // Adam steps taken
  // activations for one grid D x H x W (multiple of 8 per axis)
  int D = 0, H = 0, W = 0;
  std::vector<void*> bufs;
  float* act[CNN_NLAYER] = {};   // output of each layer (after its ReLU), cout_p channels
  float* pool[3] = {};           // avgpool2 of e1, e2, e3
  float* gact[CNN_NLAYER] = {};  // gradients with respect to layer outputs
  float* gpool[3] = {};
  float* gcat = nullptr;         // gradient of a decoder's concatenated input (largest level)
  float* x_in = nullptr;         // network input [D][H][W][16]
  float* target = nullptr;       // [D][H][W][16]
  float* wpart = nullptr;        // weight-gradient partial sums
  int64_t wpart_elems = 0;
  double* red = nullptr;         // reductions (loss, scales)
  std::vector<void*> owned;
  ~Cnn();
};

void cnn_init(Cnn& N, uint64_t seed);                         // He-normal weights, zero biases
void cnn_size(Cnn& N, int D, int H, int W);                   // allocate activations for a grid
void cnn_refresh_weights(Cnn& N, hipStream_t st);             // float32 -> bf16 GEMM layouts
void cnn_forward(Cnn& N, hipStream_t st);                     // x_in -> act[out]
// loss 0.5 sum (y - t)^2 / n into red[0] (device) and gradients of every parameter into grads
void cnn_backward(Cnn& N, hipStream_t st);
void cnn_adam(Cnn& N, float lr, hipStream_t st);

// single-layer access for the parity tests: forward of layer l on explicit buffers
void cnn_conv_forward(hipStream_t st, const float* in0, int c0, bool up0, const float* in1, int c1,
                      const float* mask, const uint16_t* w, const float* bias, bool relu, float* out, int cout_p,
                      int cout, int D, int H, int W);
void cnn_conv_wgrad(Cnn& N, hipStream_t st, int layer, const float* in0, int c0, bool up0, const float* in1, int c1,
                    const float* g, const float* mask, int cout_p, float* gw, float* gb, int D, int H, int W);

// a network with its training pairs (bfloat16 [pair][D][H][W][16]: input channels 0..7, target 8..13)
struct NetState {
  Cnn N;
  uint16_t* pairs = nullptr;
  int64_t cap = 0, count = 0;
  int D = 0, H = 0, W = 0;
  ~NetState();
};

// material channels (D^-1 of the body diagonal over its largest modulus) of a handle
void build_material(Handle& H, const std::vector<cxd>& invdiag);
// out_full's body rows += the learned correction for v_full's body part (preconditioner built)
void net_apply(Handle& H, NetState& S, const cxd* v_full, cxd* out_full, hipStream_t st);
// store the training pair of one Arnoldi step: w = A_S z (full-length vectors); dw_tmp: 3 n_v scratch
void net_collect_pair(Handle& H, NetState& S, const cxd* z_full, const cxd* w_full, cxd* dw_tmp, hipStream_t st);
// epochs of Adam over the stored pairs (shuffled, random common phase); mean loss of the last epoch
double net_train(NetState& S, int epochs, float lr, uint64_t seed, hipStream_t st);

}  // namespace vsie
