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

// ------------------------------------------------------------------ convolution
// Work is split into bricks of 4x4x4 points of one sample.  A workgroup
// stages its brick's 6x6x6 input halo (zero outside the grid) in LDS as
// BF16, so the 27 taps are LDS reads without bounds checks; wavefront w
// takes the 16 points of brick layer z = w.
constexpr int kHalo = 216;     // 6^3 halo points
constexpr int kMaxCin = 64;    // channels a halo holds

struct Brick {
  int b, x0, y0, z0;
};
__device__ __forceinline__ Brick brick_of(int64_t id, int g) {
  const int nb = (g + 3) / 4;
  Brick r;
  r.x0 = 4 * (int)(id % nb);
  r.y0 = 4 * (int)((id / nb) % nb);
  r.z0 = 4 * (int)((id / ((int64_t)nb * nb)) % nb);
  r.b = (int)(id / ((int64_t)nb * nb * nb));
  return r;
}

// halo[h * cp + c] = bf16(x[b][point of halo h][c]), cp = cin rounded up to 4
__device__ __forceinline__ void stage_halo(const float* x, const Brick& B, int g, int cin, int cp, uint16_t* halo) {
  const int64_t g3 = (int64_t)g * g * g;
  for (int i = threadIdx.x; i < kHalo * cp; i += blockDim.x) {
    const int h = i / cp, c = i - h * cp;
    const int xx = B.x0 + h % 6 - 1, yy = B.y0 + (h / 6) % 6 - 1, zz = B.z0 + h / 36 - 1;
    float v = 0.f;
    if (c < cin && xx >= 0 && yy >= 0 && zz >= 0 && xx < g && yy < g && zz < g)
      v = x[((int64_t)B.b * g3 + xx + (int64_t)g * (yy + (int64_t)g * zz)) * cin + c];
    halo[i] = to_bf16(v);
  }
}

// halo index of brick-local point (x, y, z) at tap t
__device__ __forceinline__ int halo_at(int x, int y, int z, int t) {
  return (z + t / 9) * 36 + (y + (t / 3) % 3) * 6 + (x + t % 3);
}

// y[P][co] (+)= act(sum_kk im2col(x)[P][kk] w[co][kk] + bias[co]).  MFMA
// operand layout: lane l holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) +
// j][l % 16] and D[4 (l / 16) + j][l % 16], j = 0..3; A rows are points,
// B columns output channels (up to three tiles of 16 per wavefront).
__global__ void __launch_bounds__(256) k_conv(ConvArgs a) {
  __shared__ __align__(16) uint16_t halo[kHalo * kMaxCin];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Brick B = brick_of(blockIdx.x, a.g);
  const int cp = (a.cin + 3) & ~3;
  stage_halo(a.x, B, a.g, a.cin, cp, halo);
  __syncthreads();
  const int r = lane & 15, q = lane >> 4;
  const int px = r & 3, py = r >> 2, pz = w;  // this lane's A row: brick point (px, py, pz)
  const int ntn = a.cout_pad / 16;            // 1..3
  f32x4 acc[3] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  const uint16_t* w0 = a.w + (int64_t)r * a.kpad;  // B column r of tile 0
  const int64_t tstride = (int64_t)16 * a.kpad;
  if ((a.cin & 15) == 0) {
    // every 16-column step stays inside one tap: 4 channels per lane, one 8-byte read
    for (int t = 0; t < 27; ++t) {
      const uint16_t* hp = halo + halo_at(px, py, pz, t) * cp + 4 * q;
      const int kt = t * a.cin + 4 * q;
      for (int c0 = 0; c0 < a.cin; c0 += 16) {
        const bf16x4 av = *(const bf16x4*)(hp + c0);
#pragma unroll
        for (int n = 0; n < 3; ++n)
          if (n < ntn) {
            const bf16x4 bv = *(const bf16x4*)(w0 + n * tstride + kt + c0);
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[n], 0, 0, 0);
          }
      }
    }
  } else {
    // few channels (K = 27 cin <= kpad): column kk = t cin + ci element by element
    const int K = 27 * a.cin;
    for (int k0 = 0; k0 < a.kpad; k0 += 16) {
      bf16x4 av;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = k0 + 4 * q + j;
        const int t = kk < K ? kk / a.cin : 0, ci = kk - t * a.cin;
        av[j] = kk < K ? (short)halo[halo_at(px, py, pz, t) * cp + ci] : (short)0;
      }
#pragma unroll
      for (int n = 0; n < 3; ++n)
        if (n < ntn) {
          const bf16x4 bv = *(const bf16x4*)(w0 + n * tstride + k0 + 4 * q);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[n], 0, 0, 0);
        }
    }
  }
  // D rows 4q + j are brick points (x = (4q+j) & 3, y = (4q+j) >> 2, z = w)
  const int64_t g3 = (int64_t)a.g * a.g * a.g;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    if (n >= ntn) break;
    const int co = n * 16 + r;
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * q + j;
      const int xx = B.x0 + (row & 3), yy = B.y0 + (row >> 2), zz = B.z0 + w;
      if (xx >= a.g || yy >= a.g || zz >= a.g) continue;
      float v = acc[n][j] + bias;
      if (a.relu) v = v > 0.f ? v : 0.f;
      float* dst = a.y + ((int64_t)B.b * g3 + xx + (int64_t)a.g * (yy + (int64_t)a.g * zz)) * a.cout + co;
      *dst = a.accumulate ? *dst + v : v;
    }
  }
}

// Weight gradient by chunks of bricks: part[c][co][kk] = sum over the
// points P of chunk c of dz[P][co] im2col(x)[P][kk].  MFMA with M = output
// channels, N = columns kk, inner dimension = points (one brick layer of 16
// per step).  A workgroup owns 32 (co, kk) tiles (8 per wavefront) and
// walks the bricks of its chunk, staging the input halo and dz^T in LDS.
constexpr int kWgTiles = 8;  // tiles per wavefront
__global__ void __launch_bounds__(256) k_conv_wgrad(WgradArgs a) {
  __shared__ __align__(16) uint16_t halo[kHalo * kMaxCin];
  __shared__ __align__(16) uint16_t dzt[48 * 64];  // [co][brick point]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int ntk = a.kpad / 16, ntiles = (a.cout_pad / 16) * ntk;
  const int cp = (a.cin + 3) & ~3;
  const int K = 27 * a.cin;
  const int tile0 = (blockIdx.x * 4 + w) * kWgTiles;  // this wavefront's first tile
  f32x4 acc[kWgTiles];
#pragma unroll
  for (int i = 0; i < kWgTiles; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nb = (a.g + 3) / 4;
  const int64_t nbricks = (int64_t)(a.P / ((int64_t)a.g * a.g * a.g)) * nb * nb * nb;
  const int64_t b0 = (int64_t)blockIdx.y * a.chunk, b1 = min(nbricks, b0 + a.chunk);
  const int64_t g3 = (int64_t)a.g * a.g * a.g;
  for (int64_t bid = b0; bid < b1; ++bid) {
    const Brick B = brick_of(bid, a.g);
    __syncthreads();  // the previous brick's LDS reads are done
    stage_halo(a.x, B, a.g, a.cin, cp, halo);
    for (int i = threadIdx.x; i < 64 * a.cout; i += blockDim.x) {
      const int pnt = i / a.cout, co = i - pnt * a.cout;
      const int xx = B.x0 + (pnt & 3), yy = B.y0 + ((pnt >> 2) & 3), zz = B.z0 + (pnt >> 4);
      float v = 0.f;
      if (xx < a.g && yy < a.g && zz < a.g)
        v = a.dz[((int64_t)B.b * g3 + xx + (int64_t)a.g * (yy + (int64_t)a.g * zz)) * a.cout + co];
      dzt[co * 64 + pnt] = to_bf16(v);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kWgTiles; ++i) {
      // tile (mt, kt) and this lane's column kk = t cin + ci, recomputed per
      // brick (cheap) instead of being held in registers
      const int tile = tile0 + i;
      if (tile >= ntiles) break;
      const int mt = tile / ntk, kt = tile - mt * ntk;
      const int kk = kt * 16 + r;
      const int tap = kk < K ? kk / a.cin : -1, ci = kk - (kk < K ? tap : 0) * a.cin;
      const int co = mt * 16 + r;
      for (int z = 0; z < 4; ++z) {  // 16 points per step: brick layer z
        bf16x4 av = {0, 0, 0, 0}, bv = {0, 0, 0, 0};
        if (co < a.cout) av = *(const bf16x4*)(dzt + co * 64 + 16 * z + 4 * q);
        if (tap >= 0)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int pnt = 4 * q + j;  // point (pnt & 3, pnt >> 2, z) of the brick
            bv[j] = (short)halo[halo_at(pnt & 3, pnt >> 2, z, tap) * cp + ci];
          }
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[i], 0, 0, 0);
      }
    }
  }
  float* dst = a.part + (int64_t)blockIdx.y * a.cout_pad * a.kpad;
#pragma unroll
  for (int i = 0; i < kWgTiles; ++i) {
    const int tile = tile0 + i;
    if (tile >= ntiles) break;
    const int mt = tile / ntk, kt = tile - mt * ntk;
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(int64_t)(mt * 16 + 4 * q + j) * a.kpad + kt * 16 + r] = acc[i][j];
  }
}

// grad_w[co][kk] = sum over chunks (fixed order); grad_b[co] = sum_P dz[P][co].
// gw[co][kk] = sum over chunks of part[chunk][co][kk]: 64 weights per
// workgroup, its four wavefronts taking every fourth chunk, combined in a
// fixed order (deterministic).
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* part, int nchunk, int cout, int cout_pad,
                                                      int kpad, int K, float* gw) {
  __shared__ float red[256];
  const int w = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + w;
  float s = 0.f;
  if (i < cout * K) {
    const int co = i / K, kk = i - co * K;
    for (int c = g; c < nchunk; c += 4) s += part[((int64_t)c * cout_pad + co) * kpad + kk];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && i < cout * K) gw[i] = (red[w] + red[w + 64]) + (red[w + 128] + red[w + 192]);
}
// Bias gradient in two fixed-order stages: part[blk][co] = sum of dz over
// the 256 points of block blk (tile staged in LDS, coalesced), then
// gb[co] = sum over blocks.
__global__ void __launch_bounds__(256) k_bias_part(const float* dz, int P, int cout, float* part) {
  __shared__ float tile[256 * 48];
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  for (int i = threadIdx.x; i < 256 * cout; i += 256) {
    const int64_t p = p0 + i / cout;
    tile[i] = p < P ? dz[p0 * cout + i] : 0.f;
  }
  __syncthreads();
  if ((int)threadIdx.x < cout) {
    float s = 0.f;
    for (int r = 0; r < 256; ++r) s += tile[r * cout + threadIdx.x];
    part[(int64_t)blockIdx.x * cout + threadIdx.x] = s;
  }
}
// One workgroup per channel: strided partial sums, then a fixed-order tree.
__global__ void __launch_bounds__(256) k_bias_reduce(const float* part, int nb, int cout, float* gb) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[(int64_t)b * cout + co];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
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
__global__ void k_mask_count(const float* in, int64_t n, double* part) {
  __shared__ double red[256];
  double c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += in[2 * i + 1] != 0.f ? 1.0 : 0.0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_inv_count(const double* part, int n, double* inv) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += part[i];
    *inv = c > 0 ? 1.0 / c : 0.0;
  }
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
  if (a.cin > kMaxCin || a.cout_pad > 48) return fail(HMG_ERR_UNSUPPORTED, "convolution: cin <= 64, cout <= 48");
  const int64_t nb = (a.g + 3) / 4;
  const int64_t bricks = (int64_t)(a.P / ((int64_t)a.g * a.g * a.g)) * nb * nb * nb;
  hipLaunchKernelGGL(k_conv, (unsigned)bricks, 256, 0, s, a);
  return check_launch("k_conv");
}
int net_wgrad(const WgradArgs& a, float* gw, float* gb, hipStream_t s) {
  if (a.cin > kMaxCin || a.cout_pad > 48) return fail(HMG_ERR_UNSUPPORTED, "convolution: cin <= 64, cout <= 48");
  const int ntiles = (a.cout_pad / 16) * (a.kpad / 16);
  const int per_wg = 4 * kWgTiles;
  hipLaunchKernelGGL(k_conv_wgrad, dim3((unsigned)((ntiles + per_wg - 1) / per_wg), (unsigned)a.nchunk), 256, 0, s,
                     a);
  const int K = 27 * a.cin;
  hipLaunchKernelGGL(k_wgrad_reduce, (unsigned)(((int64_t)a.cout * K + 63) / 64), 256, 0, s, a.part, a.nchunk,
                     a.cout, a.cout_pad,
                     a.kpad, K, gw);
  const unsigned nb = (unsigned)((a.P + 255) / 256);
  hipLaunchKernelGGL(k_bias_part, nb, 256, 0, s, a.dz, a.P, a.cout, a.bpart);
  hipLaunchKernelGGL(k_bias_reduce, (unsigned)a.cout, 256, 0, s, a.bpart, (int)nb, a.cout, gb);
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
  // partials[nparts] holds 1 / count (the partials are reused for the loss)
  hipLaunchKernelGGL(k_mask_count, nparts, 256, 0, s, in, n, partials);
  hipLaunchKernelGGL(k_inv_count, 1, 64, 0, s, partials, nparts, partials + nparts);
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
