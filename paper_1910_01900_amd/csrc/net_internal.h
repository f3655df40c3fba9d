// Internal declarations of the learned coarse-grid correction: kernel
// argument blocks, launchers and the network handle.
#pragma once

#include "hmg_internal.h"

namespace hmg {

// Implicit-GEMM convolution y[P][co] = act(sum_kk im2col(x)[P][kk] w[co][kk]
// + bias[co]) over P = B g^3 points (channels-last activations, FP32),
// kk = t cin + ci for the 27 taps t of a 3x3x3 stencil with zero padding.
struct ConvArgs {
  const float* x;
  const uint16_t* w;  // BF16 [cout_pad][kpad], zero-padded
  const float* bias;  // [cout] or NULL
  float* y;
  int P, g, cin, cout, cout_pad, kpad;
  int relu, accumulate;  // y = relu(..) ; y += .. instead of y = ..
};
// Weight gradient by chunks of 4x4x4-point bricks: part[c][co][kk]
// (cout_pad x kpad per chunk of `chunk` bricks).
struct WgradArgs {
  const float* x;   // layer input [P][cin]
  const float* dz;  // gradient of the layer's pre-activation [P][cout]
  float* part;
  float* bpart;  // bias partials: ceil(P / 256) x cout
  int P, g, cin, cout, cout_pad, kpad, chunk, nchunk;
};
// 4x4x4-point bricks of `batch` samples on a g^3 grid
inline int64_t net_bricks(int64_t batch, int g) {
  const int64_t nb = (g + 3) / 4;
  return batch * nb * nb * nb;
}

int net_conv(const ConvArgs& a, hipStream_t s);
int net_wgrad(const WgradArgs& a, float* gw, float* gb, hipStream_t s);
int net_weight_prep(const float* w, int cin, int cout, uint16_t* wf, int cout_pad, int kpad_f, uint16_t* wt,
                    int cin_pad, int kpad_t, hipStream_t s);
int net_pool(const float* x, float* y, int B, int g, int c, hipStream_t s);
int net_pool_bwd(const float* dy, float* dx, int B, int g, int c, int acc, hipStream_t s);
int net_up_add(const float* a, const float* sk, float* u, int B, int g, int c, hipStream_t s);
int net_up_bwd(const float* du, float* da, int B, int g, int c, hipStream_t s);
int net_relu_bwd(const float* a, const float* da, float* dz, int64_t n, hipStream_t s);
int net_copy(const float* x, float* y, int64_t n, hipStream_t s);
// Masked MSE (mean over the points whose input mask is set): *loss and
// dout; partials holds nparts + 1 doubles.
int net_mse(const float* out, const float* tgt, const float* in, int B, int g3, float* dout, double* partials,
            int nparts, double* loss, hipStream_t s);
int net_adam(float* w, const float* gw, float* m, float* v, int64_t n, float lr_t, float b1, float b2, float eps,
             hipStream_t s);

// Nodes of a continuous Q1..Qk level on a box: Mx x My x Mz nodes,
// lexicographic; a node on a face without the Neumann bit is constrained.
struct NodeGrid {
  int Mx, My, Mz, bcmask;
};
// Network input / target from coarse vectors r_b, e_b (b < B, stride ld):
// in[b][p] = (r_b(node p) / sigma_b, mask(p)), tgt[b][p] = e_b(node p) /
// (sigma_b c0), sigma_b the RMS of r_b over the free nodes (1 if zero);
// points of the G^3 grid without a node and constrained nodes are 0 / mask 0.
int net_pack(int prec, const void* r, const void* e, int64_t ld, int B, const NodeGrid& ng, int G, double c0,
             double* sigma, float* in, float* tgt, hipStream_t s);
// x(node) = out[p] sigma c0 on free nodes, 0 on constrained nodes (one sample).
int net_unpack(int prec, const float* out, const NodeGrid& ng, int G, const double* sigma, double c0, void* x,
               hipStream_t s);
// E[s][i] = sum_j Ainv[i][j] R[s][j] (FP64, count samples of n values).
int coarse_gemm(const double* Ainv, const double* R, double* E, int n, int count, hipStream_t s);
// x = Ainv b unless gate = (|b - A x|^2, |b|^2) shows |b - A x| <= accept |b|
// (finite); each fallback adds one to *fallbacks.
int coarse_gemv_gated(int prec, const double* Ainv, const void* b, void* x, int n, const double* gate,
                      double accept, int* fallbacks, hipStream_t s);

}  // namespace hmg

// ---------------------------------------------------------------- network handle
// U-Net on a G^3 grid (G divisible by 8), channels-last FP32 activations,
// 4 levels (G, G/2, G/4, G/8), 2x2x2 average pooling down, nearest
// upsampling plus skip addition up:
//   L0 2->16, L1 16->16 (G); L2 16->32 (G/2); L3 32->48 (G/4); L4 48->48 (G/8);
//   L5 48->32 (G/4); L6 32->16 (G/2); L7 16->1 (G, linear); ReLU elsewhere.
// Parameters (FP32, packed): per layer w[cout][27][cin] then b[cout].
namespace hmg {
constexpr int kNetLayers = 8;
struct NetLayer {
  int cin, cout, level, relu;
  int64_t off_w, off_b;  // into the parameter vector
  int cout_pad, kpad_f, cin_pad, kpad_t;
  size_t off_wf, off_wt;  // BF16 matrices (bytes into the workspace)
};
}  // namespace hmg

struct hmg_net {
  int G = 16, max_batch = 1;
  uint64_t seed = 1;
  hmg::NetLayer L[hmg::kNetLayers];
  int64_t n_params = 0;
  int64_t step = 0;     // Adam steps taken
  int64_t version = 0;  // changes whenever the parameters do
  bool dirty = true;  // BF16 matrices out of date
  size_t ws_bytes = 0;
  char* ws = nullptr;
  bool bound = false;
  // workspace offsets (bytes)
  size_t off_w = 0, off_g = 0, off_m = 0, off_v = 0, off_part = 0, off_bpart = 0, off_lpart = 0, off_loss = 0;
  size_t off_act[16] = {}, off_grad[16] = {};
  size_t off_hin = 0, off_hout = 0, off_hsig = 0;
  int64_t part_floats = 0;
  float* f(size_t off) const { return (float*)(ws + off); }
};

namespace hmg {
// BF16 weight matrices from the current parameters (if out of date).
int net_prepare(hmg_net* N, hipStream_t s);
// Forward pass of `batch` samples (in [batch][G^3][2] -> out [batch][G^3]).
int net_forward(hmg_net* N, const float* in, float* out, int batch, hipStream_t s);
// Single-sample buffers used by the multigrid coarse level.
inline float* net_hin(const hmg_net* N) { return N->f(N->off_hin); }
inline float* net_hout(const hmg_net* N) { return N->f(N->off_hout); }
inline double* net_hsigma(const hmg_net* N) { return (double*)(N->ws + N->off_hsig); }
}  // namespace hmg
