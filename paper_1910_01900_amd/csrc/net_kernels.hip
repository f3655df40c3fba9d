// Kernels of the learned coarse-grid correction: a small 3-D convolutional
// network on the nodes of the coarsest continuous Q1 level, trained and run
// on the GPU.  Convolutions (3x3x3, zero padding, channels-last activations)
// are implicit GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation); pooling, upsampling, the loss, Adam and the exchange
// with the multigrid hierarchy are plain FP32/FP64 kernels.
#include "net_internal.h"

namespace hmg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Neighbour of point p (index inside one sample's g^3 grid, x fastest) at
// tap t = (dx+1) + 3 (dy+1) + 9 (dz+1); -1 outside the grid.
__device__ __forceinline__ int tap_point(int p, int t, int g) {
  const int x = p % g, y = (p / g) % g, z = p / (g * g);
  const int xx = x + t % 3 - 1, yy = y + (t / 3) % 3 - 1, zz = z + t / 9 - 1;
  if (xx < 0 || yy < 0 || zz < 0 || xx >= g || yy >= g || zz >= g) return -1;
  return xx + g * (yy + g * zz);
}

// Column kk = t cin + ci of the implicit im2col matrix at point P (global
// index b g^3 + p): x[neighbour][ci], 0 outside the grid or past K.
__device__ __forceinline__ float im2col(const float* x, int P, int kk, int K, int cin, int g) {
  if (kk >= K) return 0.f;
  const int t = kk / cin, ci = kk - t * cin;
  const int g3 = g * g * g, b = P / g3, p = P - b * g3;
  const int q = tap_point(p, t, g);
  return q < 0 ? 0.f : x[((int64_t)b * g3 + q) * cin + ci];
}

// ------------------------------------------------------------------ convolution
// y[P][co] (+)= act(sum_kk im2col(x)[P][kk] w[co][kk] + bias[co]).  One
// wavefront computes 16 points x 16 output channels; the MFMA operand
// layout: lane l holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16]
// and D[4 (l / 16) + j][l % 16], j = 0..3.
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ntn = a.cout_pad / 16;
  const int64_t npt = ((int64_t)a.P + 15) / 16;
  if (wid >= npt * ntn) return;
  const int pt = (int)(wid / ntn), nt = (int)(wid - (int64_t)pt * ntn);
  const int r = lane & 15, kq = 4 * (lane >> 4);
  const int P = pt * 16 + r;  // this lane's A row
  const int K = 27 * a.cin;
  const uint16_t* wrow = a.w + (int64_t)(nt * 16 + r) * a.kpad;  // this lane's B column
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < a.kpad; k0 += 16) {
    bf16x4 av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = P < a.P ? im2col(a.x, P, k0 + kq + j, K, a.cin, a.g) : 0.f;
      av[j] = (short)to_bf16(v);
      bv[j] = (short)wrow[k0 + kq + j];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  const int co = nt * 16 + r;
  if (co >= a.cout) return;
  const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int Pj = pt * 16 + kq + j;
    if (Pj >= a.P) continue;
    float v = acc[j] + bias;
    if (a.relu) v = v > 0.f ? v : 0.f;
    float* dst = a.y + (int64_t)Pj * a.cout + co;
    *dst = a.accumulate ? *dst + v : v;
  }
}

// Weight gradient, split over point chunks: part[c][co][kk] =
// sum_{P in chunk c} dz[P][co] im2col(x)[P][kk].  MFMA with M = output
// channels, N = columns kk, inner dimension = points.
__global__ void __launch_bounds__(256) k_conv_wgrad(WgradArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ntm = a.cout_pad / 16, ntk = a.kpad / 16;
  const int64_t per_chunk = (int64_t)ntm * ntk;
  if (wid >= per_chunk * a.nchunk) return;
  const int c = (int)(wid / per_chunk);
  const int rem = (int)(wid - (int64_t)c * per_chunk);
  const int mt = rem / ntk, kt = rem - mt * ntk;
  const int r = lane & 15, pq = 4 * (lane >> 4);
  const int K = 27 * a.cin;
  const int co_a = mt * 16 + r;  // A row (output channel)
  const int kk_b = kt * 16 + r;  // B column
  const int p0 = c * a.chunk, p1 = min(a.P, p0 + a.chunk);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int pb = p0; pb < p1; pb += 16) {
    bf16x4 av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int Pj = pb + pq + j;
      const bool in = Pj < p1;
      av[j] = (short)to_bf16(in && co_a < a.cout ? a.dz[(int64_t)Pj * a.cout + co_a] : 0.f);
      bv[j] = (short)to_bf16(in ? im2col(a.x, Pj, kk_b, K, a.cin, a.g) : 0.f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  float* dst = a.part + (int64_t)c * a.cout_pad * a.kpad;
#pragma unroll
  for (int j = 0; j < 4; ++j) dst[(int64_t)(mt * 16 + pq + j) * a.kpad + kt * 16 + r] = acc[j];
}

// grad_w[co][kk] = sum over chunks (fixed order); grad_b[co] = sum_P dz[P][co].
__global__ void k_wgrad_reduce(const float* part, int nchunk, int cout, int cout_pad, int kpad, int K,
                               float* gw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cout * K) return;
  const int co = i / K, kk = i - co * K;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[((int64_t)c * cout_pad + co) * kpad + kk];
  gw[i] = s;
}
__global__ void k_bias_grad(const float* dz, int P, int cout, float* gb) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int p = threadIdx.x; p < P; p += blockDim.x) s += dz[(int64_t)p * cout + co];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) gb[co] = red[0];
}

// BF16 weight matrices from the FP32 parameters w[co][t][ci]:
// forward wf[co][t cin + ci] = w[co][t][ci], transposed-flipped (data
// gradient as a convolution of dz) wt[ci][t cout + co] = w[co][26 - t][ci];
// both zero-padded to 16 rows and kpad columns.
__global__ void k_weight_prep(const float* w, int cin, int cout, uint16_t* wf, int cout_pad, int kpad_f,
                              uint16_t* wt, int cin_pad, int kpad_t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = cout_pad * kpad_f, nt = cin_pad * kpad_t;
  if (i < nf) {
    const int co = i / kpad_f, kk = i - co * kpad_f;
    float v = 0.f;
    if (co < cout && kk < 27 * cin) v = w[(int64_t)co * 27 * cin + kk];
    wf[i] = to_bf16(v);
  } else if (wt && i < nf + nt) {
    const int j = i - nf, ci = j / kpad_t, kk = j - ci * kpad_t;
    float v = 0.f;
    if (ci < cin && kk < 27 * cout) {
      const int t = kk / cout, co = kk - t * cout;
      v = w[((int64_t)co * 27 + (26 - t)) * cin + ci];
    }
    wt[j] = to_bf16(v);
  }
}

// ------------------------------------------------------------------ elementwise
// 2x2x2 average pooling: y (grid g/2) from x (grid g), c channels.
__global__ void k_pool(const float* x, float* y, int B, int g, int c) {
  const int h = g / 2;
  const int64_t n = (int64_t)B * h * h * h * c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ch = (int)(i % c);
  int64_t q = i / c;
  const int X = (int)(q % h), Y = (int)((q / h) % h), Z = (int)((q / ((int64_t)h * h)) % h);
  const int64_t b = q / ((int64_t)h * h * h);
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int xx = 2 * X + (d & 1), yy = 2 * Y + ((d >> 1) & 1), zz = 2 * Z + (d >> 2);
    s += x[((b * g + zz) * g + yy) * (int64_t)g * c + (int64_t)xx * c + ch];
  }
  y[i] = 0.125f * s;
}
// dx (+)= dy / 8 spread to the 8 children (dx on grid g, dy on g/2).
__global__ void k_pool_bwd(const float* dy, float* dx, int B, int g, int c, int accumulate) {
  const int64_t n = (int64_t)B * g * g * g * c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int h = g / 2, ch = (int)(i % c);
  int64_t q = i / c;
  const int x = (int)(q % g), y = (int)((q / g) % g), z = (int)((q / ((int64_t)g * g)) % g);
  const int64_t b = q / ((int64_t)g * g * g);
  const float v = 0.125f * dy[(((b * h + z / 2) * h + y / 2) * h + x / 2) * c + ch];
  dx[i] = accumulate ? dx[i] + v : v;
}
// u (grid g) = nearest upsampling of a (grid g/2) + s (grid g).
__global__ void k_up_add(const float* a, const float* s, float* u, int B, int g, int c) {
  const int64_t n = (int64_t)B * g * g * g * c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int h = g / 2, ch = (int)(i % c);
  int64_t q = i / c;
  const int x = (int)(q % g), y = (int)((q / g) % g), z = (int)((q / ((int64_t)g * g)) % g);
  const int64_t b = q / ((int64_t)g * g * g);
  u[i] = a[(((b * h + z / 2) * h + y / 2) * h + x / 2) * c + ch] + s[i];
}
// da (grid g/2) = sum of du over the 8 children (du on grid g).
__global__ void k_up_bwd(const float* du, float* da, int B, int g, int c) {
  const int h = g / 2;
  const int64_t n = (int64_t)B * h * h * h * c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ch = (int)(i % c);
  int64_t q = i / c;
  const int X = (int)(q % h), Y = (int)((q / h) % h), Z = (int)((q / ((int64_t)h * h)) % h);
  const int64_t b = q / ((int64_t)h * h * h);
  float s = 0.f;
  for (int d = 0; d < 8; ++d) {
    const int xx = 2 * X + (d & 1), yy = 2 * Y + ((d >> 1) & 1), zz = 2 * Z + (d >> 2);
    s += du[((b * g + zz) * g + yy) * (int64_t)g * c + (int64_t)xx * c + ch];
  }
  da[i] = s;
}
// dz = da where a > 0 (a: ReLU output), else 0; in place allowed.
__global__ void k_relu_bwd(const float* a, const float* da, float* dz, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = a[i] > 0.f ? da[i] : 0.f;
}
__global__ void k_copy_f(const float* x, float* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// Masked mean squared error over B samples of g^3 points, averaged over
// the points whose input mask (channel 1) is set: loss partials and
// d loss / d out = 2 mask (out - t) / count.
__global__ void k_mask_count(const float* in, int64_t n, double* inv_count) {
  __shared__ double red[1024];
  double c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) c += in[2 * i + 1] != 0.f ? 1.0 : 0.0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *inv_count = red[0] > 0 ? 1.0 / red[0] : 0.0;
}
__global__ void k_mse(const float* out, const float* tgt, const float* in, int64_t n, const double* inv_count,
                      float* dout, double* partials) {
  __shared__ double red[256];
  const double inv = *inv_count;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float m = in[2 * i + 1];
    const float d = m * (out[i] - tgt[i]);
    dout[i] = (float)(2.0 * d * inv);
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] * inv;
}
__global__ void k_sum_partials(const double* p, int n, double* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    *out = s;
  }
}

// Adam (Kingma and Ba 2015) with bias-corrected step size lr_t.
__global__ void k_adam(float* w, const float* gw, float* m, float* v, int64_t n, float lr_t, float b1, float b2,
                       float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gw[i];
  const float mi = b1 * m[i] + (1.f - b1) * g, vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr_t * mi / (sqrtf(vi) + eps);
}

// ------------------------------------------------------------------ launchers
static unsigned blocks(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

int net_conv(const ConvArgs& a, hipStream_t s) {
  const int64_t waves = ((int64_t)a.P + 15) / 16 * (a.cout_pad / 16);
  hipLaunchKernelGGL(k_conv, blocks(waves, 4), 256, 0, s, a);
  return check_launch("k_conv");
}
int net_wgrad(const WgradArgs& a, float* gw, float* gb, hipStream_t s) {
  const int64_t waves = (int64_t)(a.cout_pad / 16) * (a.kpad / 16) * a.nchunk;
  hipLaunchKernelGGL(k_conv_wgrad, blocks(waves, 4), 256, 0, s, a);
  const int K = 27 * a.cin;
  hipLaunchKernelGGL(k_wgrad_reduce, blocks((int64_t)a.cout * K), 256, 0, s, a.part, a.nchunk, a.cout, a.cout_pad,
                     a.kpad, K, gw);
  hipLaunchKernelGGL(k_bias_grad, a.cout, 256, 0, s, a.dz, a.P, a.cout, gb);
  return check_launch("k_conv_wgrad");
}
int net_weight_prep(const float* w, int cin, int cout, uint16_t* wf, int cout_pad, int kpad_f, uint16_t* wt,
                    int cin_pad, int kpad_t, hipStream_t s) {
  const int64_t n = (int64_t)cout_pad * kpad_f + (wt ? (int64_t)cin_pad * kpad_t : 0);
  hipLaunchKernelGGL(k_weight_prep, blocks(n), 256, 0, s, w, cin, cout, wf, cout_pad, kpad_f, wt, cin_pad, kpad_t);
  return check_launch("k_weight_prep");
}
int net_pool(const float* x, float* y, int B, int g, int c, hipStream_t s) {
  const int h = g / 2;
  hipLaunchKernelGGL(k_pool, blocks((int64_t)B * h * h * h * c), 256, 0, s, x, y, B, g, c);
  return check_launch("k_pool");
}
int net_pool_bwd(const float* dy, float* dx, int B, int g, int c, int acc, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd, blocks((int64_t)B * g * g * g * c), 256, 0, s, dy, dx, B, g, c, acc);
  return check_launch("k_pool_bwd");
}
int net_up_add(const float* a, const float* sk, float* u, int B, int g, int c, hipStream_t s) {
  hipLaunchKernelGGL(k_up_add, blocks((int64_t)B * g * g * g * c), 256, 0, s, a, sk, u, B, g, c);
  return check_launch("k_up_add");
}
int net_up_bwd(const float* du, float* da, int B, int g, int c, hipStream_t s) {
  const int h = g / 2;
  hipLaunchKernelGGL(k_up_bwd, blocks((int64_t)B * h * h * h * c), 256, 0, s, du, da, B, g, c);
  return check_launch("k_up_bwd");
}
int net_relu_bwd(const float* a, const float* da, float* dz, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_bwd, blocks(n), 256, 0, s, a, da, dz, n);
  return check_launch("k_relu_bwd");
}
int net_copy(const float* x, float* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f, blocks(n), 256, 0, s, x, y, n);
  return check_launch("k_copy_f");
}
int net_mse(const float* out, const float* tgt, const float* in, int B, int g3, float* dout, double* partials,
            int nparts, double* loss, hipStream_t s) {
  const int64_t n = (int64_t)B * g3;
  // partials[nparts] holds 1 / count
  hipLaunchKernelGGL(k_mask_count, 1, 1024, 0, s, in, n, partials + nparts);
  hipLaunchKernelGGL(k_mse, nparts, 256, 0, s, out, tgt, in, n, (const double*)(partials + nparts), dout, partials);
  hipLaunchKernelGGL(k_sum_partials, 1, 64, 0, s, partials, nparts, loss);
  return check_launch("k_mse");
}
int net_adam(float* w, const float* gw, float* m, float* v, int64_t n, float lr_t, float b1, float b2, float eps,
             hipStream_t s) {
  hipLaunchKernelGGL(k_adam, blocks(n), 256, 0, s, w, gw, m, v, n, lr_t, b1, b2, eps);
  return check_launch("k_adam");
}

}  // namespace hmg

namespace hmg {

// ------------------------------------------------------------------ hierarchy exchange
__device__ __forceinline__ bool node_of(int p, int G, const NodeGrid& ng, int64_t* node, bool* freeN) {
  const int x = p % G, y = (p / G) % G, z = p / (G * G);
  if (x >= ng.Mx || y >= ng.My || z >= ng.Mz) return false;
  *node = x + (int64_t)ng.Mx * (y + (int64_t)ng.My * z);
  const int m = ng.bcmask;
  const bool fixed = (x == 0 && !(m & 1)) || (x == ng.Mx - 1 && !(m & 2)) || (y == 0 && !(m & 4)) ||
                     (y == ng.My - 1 && !(m & 8)) || (z == 0 && !(m & 16)) || (z == ng.Mz - 1 && !(m & 32));
  *freeN = !fixed;
  return true;
}

// sigma_b = RMS of r_b over the free nodes (1 when zero); one block per sample.
template <typename T>
__global__ void k_sample_rms(const T* r, int64_t ld, NodeGrid ng, int G, double* sigma) {
  __shared__ double red[256], cnt[256];
  const int b = blockIdx.x;
  double s = 0.0, c = 0.0;
  for (int p = threadIdx.x; p < G * G * G; p += blockDim.x) {
    int64_t node;
    bool fr;
    if (node_of(p, G, ng, &node, &fr) && fr) {
      const double v = (double)r[(int64_t)b * ld + node];
      s += v * v;
      c += 1.0;
    }
  }
  red[threadIdx.x] = s;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[threadIdx.x] += red[threadIdx.x + o];
      cnt[threadIdx.x] += cnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double rms = cnt[0] > 0 ? sqrt(red[0] / cnt[0]) : 0.0;
    sigma[b] = rms > 0 && isfinite(rms) ? rms : 1.0;
  }
}

template <typename T>
__global__ void k_net_pack(const T* r, const T* e, int64_t ld, int B, NodeGrid ng, int G, double c0,
                           const double* sigma, float* in, float* tgt) {
  const int64_t n = (int64_t)B * G * G * G;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)(i / (G * G * G)), p = (int)(i - (int64_t)b * G * G * G);
  int64_t node = 0;
  bool fr = false;
  const bool has = node_of(p, G, ng, &node, &fr) && fr;
  const double sg = sigma[b];
  in[2 * i] = has ? (float)((double)r[(int64_t)b * ld + node] / sg) : 0.f;
  in[2 * i + 1] = has ? 1.f : 0.f;
  if (tgt) tgt[i] = has ? (float)((double)e[(int64_t)b * ld + node] / (sg * c0)) : 0.f;
}

template <typename T>
__global__ void k_net_unpack(const float* out, NodeGrid ng, int G, const double* sigma, double c0, T* x) {
  const int64_t nn = (int64_t)ng.Mx * ng.My * ng.Mz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int xx = (int)(i % ng.Mx), yy = (int)((i / ng.Mx) % ng.My), zz = (int)(i / ((int64_t)ng.Mx * ng.My));
  int64_t node;
  bool fr;
  node_of(xx + G * (yy + G * zz), G, ng, &node, &fr);
  x[i] = fr ? (T)((double)out[xx + G * (yy + G * zz)] * sigma[0] * c0) : T(0);
}

int net_pack(int prec, const void* r, const void* e, int64_t ld, int B, const NodeGrid& ng, int G, double c0,
             double* sigma, float* in, float* tgt, hipStream_t s) {
  const int64_t n = (int64_t)B * G * G * G;
  if (prec == HMG_F64) {
    hipLaunchKernelGGL(k_sample_rms<double>, B, 256, 0, s, (const double*)r, ld, ng, G, sigma);
    hipLaunchKernelGGL(k_net_pack<double>, blocks(n), 256, 0, s, (const double*)r, (const double*)e, ld, B, ng, G,
                       c0, (const double*)sigma, in, tgt);
  } else {
    hipLaunchKernelGGL(k_sample_rms<float>, B, 256, 0, s, (const float*)r, ld, ng, G, sigma);
    hipLaunchKernelGGL(k_net_pack<float>, blocks(n), 256, 0, s, (const float*)r, (const float*)e, ld, B, ng, G, c0,
                       (const double*)sigma, in, tgt);
  }
  return check_launch("net_pack");
}

int net_unpack(int prec, const float* out, const NodeGrid& ng, int G, const double* sigma, double c0, void* x,
               hipStream_t s) {
  const int64_t nn = (int64_t)ng.Mx * ng.My * ng.Mz;
  if (prec == HMG_F64)
    hipLaunchKernelGGL(k_net_unpack<double>, blocks(nn), 256, 0, s, out, ng, G, sigma, c0, (double*)x);
  else
    hipLaunchKernelGGL(k_net_unpack<float>, blocks(nn), 256, 0, s, out, ng, G, sigma, c0, (float*)x);
  return check_launch("net_unpack");
}

// E = R Ainv^T (= R Ainv, Ainv symmetric): 64 x 64 output tiles, LDS-staged
// 64 x 16 slices of R and Ainv, 4 x 4 outputs per thread.
__global__ void __launch_bounds__(256) k_coarse_gemm(const double* A, const double* R, double* E, int n, int count) {
  __shared__ double Rs[64][17], As[64][17];
  const int s0 = blockIdx.y * 64, i0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int j0 = 0; j0 < n; j0 += 16) {
    for (int q = threadIdx.x; q < 64 * 16; q += 256) {
      const int rr = q / 16, cc = q % 16;
      const int sj = s0 + rr, ij = i0 + rr, jj = j0 + cc;
      Rs[rr][cc] = (sj < count && jj < n) ? R[(int64_t)sj * n + jj] : 0.0;
      As[rr][cc] = (ij < n && jj < n) ? A[(int64_t)ij * n + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += Rs[ty + 16 * a][c] * As[tx + 16 * b][c];
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int sj = s0 + ty + 16 * a, ij = i0 + tx + 16 * b;
      if (sj < count && ij < n) E[(int64_t)sj * n + ij] = acc[a][b];
    }
}

int coarse_gemm(const double* Ainv, const double* R, double* E, int n, int count, hipStream_t s) {
  if (n <= 0 || count <= 0) return HMG_OK;
  dim3 g((unsigned)((n + 63) / 64), (unsigned)((count + 63) / 64));
  hipLaunchKernelGGL(k_coarse_gemm, g, 256, 0, s, Ainv, R, E, n, count);
  return check_launch("coarse_gemm");
}

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_gemv_gated(const double* Ainv, const T* b, T* x, int n,
                                                           const double* gate, double accept2, int* fallbacks) {
  const double rr = gate[0], bb = gate[1];
  if (isfinite(rr) && rr <= accept2 * bb) return;  // the network's correction is kept
  if (blockIdx.x == 0 && threadIdx.x == 0) fallbacks[0] += 1;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* Ar = Ainv + (int64_t)row * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += Ar[j] * (double)b[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[row] = (T)acc;
}

int coarse_gemv_gated(int prec, const double* Ainv, const void* b, void* x, int n, const double* gate,
                      double accept, int* fallbacks, hipStream_t s) {
  const unsigned g = (unsigned)((n + 3) / 4);
  const double a2 = accept * accept;
  if (prec == HMG_F64)
    hipLaunchKernelGGL(k_coarse_gemv_gated<double>, g, 256, 0, s, Ainv, (const double*)b, (double*)x, n, gate, a2,
                       fallbacks);
  else
    hipLaunchKernelGGL(k_coarse_gemv_gated<float>, g, 256, 0, s, Ainv, (const float*)b, (float*)x, n, gate, a2,
                       fallbacks);
  return check_launch("coarse_gemv_gated");
}

}  // namespace hmg
