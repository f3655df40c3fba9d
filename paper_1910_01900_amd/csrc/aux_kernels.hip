// Vector operations, deterministic reductions, CG updates, FE node sums,
// multigrid transfers and the coarse-level dense solve for gfx950.
#include "hmg_internal.h"

#include <algorithm>

namespace hmg {

static constexpr int kBlock = 256;

static unsigned grid_for(int64_t n, int per_thread = 4) {
  int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
  if (g < 1) g = 1;
  if (g > 65535 * 8) g = 65535 * 8;
  return (unsigned)g;
}

__device__ __forceinline__ double block_reduce(double v) {
  __shared__ double red[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// ------------------------------------------------------------------ elementwise
template <typename T>
__global__ void k_fill(T* x, T a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = a;
}
template <typename T>
__global__ void k_axpby(T a, const T* x, T b, const T* y, T* z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = a * x[i] + (y ? b * y[i] : T(0));
}
template <typename T>
__global__ void k_recip(const T* x, T* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = T(1) / x[i];
}
template <typename T>
__global__ void k_mul3(T a, const T* d, const T* b, T* z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = a * d[i] * b[i];
}
template <typename A, typename B>
__global__ void k_convert(const A* x, B* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (B)x[i];
}
// y = x converted, skipped while *skip != 0 (gated coarse solves)
template <typename A, typename B>
__global__ void k_convert_gated(const A* x, B* y, int64_t n, const int* skip) {
  if (*skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (B)x[i];
}
template <typename T>
__global__ void k_dot(const T* x, const T* y, int64_t n, double* partials) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
__global__ void k_reduce(const double* partials, int np, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) *out = s;
}
// Block (b, r): tmp[r * gridDim.x + b] = sum over j = b * blockDim.x + t
// + k * gridDim.x * blockDim.x < n of partials[r + nrhs * j] (per-thread
// sums in a fixed order, then the block's fixed tree); k_reduce_b then sums
// each vector's gridDim.x values.
__global__ void k_reduce_strided(const double* partials, int64_t n, int nrhs, double* tmp) {
  const int r = blockIdx.y;
  double acc = 0.0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    acc += partials[r + (int64_t)nrhs * j];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) tmp[r * gridDim.x + blockIdx.x] = s;
}
// SplitMix64 (Steele, Lea, Flood 2014): output i = mix(seed + (i+1)*golden)
template <typename T>
__global__ void k_splitmix(uint64_t seed, T* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (T)((double)(z >> 11) * 0x1.0p-52 - 1.0);
  }
}

// CG (Alg. 1): omega = delta / (p^T v); x += omega p; r -= omega v; partials of r.r
__global__ void k_cg_xr(double* x, double* r, const double* p, const double* v, const double* num,
                        const double* den, int64_t n, double* partials, double* save, float* r32) {
  const double omega = *num / *den;
  // keep delta = *num for the next iteration's beta (save != num, den)
  if (save && blockIdx.x == 0 && threadIdx.x == 0) *save = *num;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += omega * p[i];
    const double ri = r[i] - omega * v[i];
    r[i] = ri;
    if (r32) r32[i] = (float)ri;  // the next V-cycle's FP32 right-hand side
    acc += ri * ri;
  }
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
// partials of x . z with z in FP32 (widened exactly), as k_dot
__global__ void k_dot_zf(const double* x, const float* z, int64_t n, double* partials) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * (double)z[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
// p = z + (*num / *den) p with z in FP32; den = NULL: p = z
__global__ void k_cg_p_zf(double* p, const float* z, const double* num, const double* den, int64_t n) {
  const double beta = den ? *num / *den : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = den ? (double)z[i] + beta * p[i] : (double)z[i];
}
// p = z + beta p, beta = (+-) *num / *den
__global__ void k_cg_p(double* p, const double* z, const double* num, const double* den, int64_t n, int neg) {
  const double beta = (neg ? -*num : *num) / *den;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

#define PREC_DISPATCH(prec, EXPR_D, EXPR_F) \
  do {                                      \
    if ((prec) == HMG_F64) {                \
      EXPR_D;                               \
    } else {                                \
      EXPR_F;                               \
    }                                       \
  } while (0)

int vec_fill(int prec, void* x, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  PREC_DISPATCH(prec, hipLaunchKernelGGL(k_fill<double>, grid_for(n), kBlock, 0, s, (double*)x, a, n),
                hipLaunchKernelGGL(k_fill<float>, grid_for(n), kBlock, 0, s, (float*)x, (float)a, n));
  return check_launch("fill");
}
int vec_copy(int prec, const void* x, void* y, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  HMG_HIP(hipMemcpyAsync(y, x, (size_t)n * (prec == HMG_F64 ? 8 : 4), hipMemcpyDeviceToDevice, s));
  return HMG_OK;
}
int vec_axpby(int prec, double a, const void* x, double b, const void* y, void* z, int64_t n,
              hipStream_t s) {
  if (n <= 0) return HMG_OK;
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_axpby<double>, grid_for(n), kBlock, 0, s, a, (const double*)x, b,
                                   (const double*)y, (double*)z, n),
                hipLaunchKernelGGL(k_axpby<float>, grid_for(n), kBlock, 0, s, (float)a, (const float*)x,
                                   (float)b, (const float*)y, (float*)z, n));
  return check_launch("axpby");
}
int vec_recip(int prec, const void* x, void* y, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  PREC_DISPATCH(prec, hipLaunchKernelGGL(k_recip<double>, grid_for(n), kBlock, 0, s, (const double*)x, (double*)y, n),
                hipLaunchKernelGGL(k_recip<float>, grid_for(n), kBlock, 0, s, (const float*)x, (float*)y, n));
  return check_launch("recip");
}
int vec_mul3(int prec, double a, const void* d, const void* b, void* z, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_mul3<double>, grid_for(n), kBlock, 0, s, a, (const double*)d,
                                   (const double*)b, (double*)z, n),
                hipLaunchKernelGGL(k_mul3<float>, grid_for(n), kBlock, 0, s, (float)a, (const float*)d,
                                   (const float*)b, (float*)z, n));
  return check_launch("mul3");
}
int vec_convert(int from, const void* x, int to, void* y, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  if (from == to) return vec_copy(from, x, y, n, s);
  if (from == HMG_F64)
    hipLaunchKernelGGL((k_convert<double, float>), grid_for(n), kBlock, 0, s, (const double*)x, (float*)y, n);
  else
    hipLaunchKernelGGL((k_convert<float, double>), grid_for(n), kBlock, 0, s, (const float*)x, (double*)y, n);
  return check_launch("convert");
}
int vec_convert_gated(int from, const void* x, int to, void* y, int64_t n, const int* skip, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  if (from == HMG_F64 && to == HMG_F64)
    hipLaunchKernelGGL((k_convert_gated<double, double>), grid_for(n), kBlock, 0, s, (const double*)x, (double*)y, n, skip);
  else if (from == HMG_F64)
    hipLaunchKernelGGL((k_convert_gated<double, float>), grid_for(n), kBlock, 0, s, (const double*)x, (float*)y, n, skip);
  else if (to == HMG_F64)
    hipLaunchKernelGGL((k_convert_gated<float, double>), grid_for(n), kBlock, 0, s, (const float*)x, (double*)y, n, skip);
  else
    hipLaunchKernelGGL((k_convert_gated<float, float>), grid_for(n), kBlock, 0, s, (const float*)x, (float*)y, n, skip);
  return check_launch("convert_gated");
}
static unsigned dot_grid(int64_t n) {
  unsigned g = grid_for(n, 8);
  return g > (unsigned)kPartials ? (unsigned)kPartials : g;
}
int reduce_partials(const double* partials, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, 1, 1024, 0, s, partials, np, out);
  return check_launch("reduce");
}
int vec_dot(int prec, const void* x, const void* y, int64_t n, double* partials, double* out,
            hipStream_t s) {
  const unsigned g = dot_grid(n);
  PREC_DISPATCH(prec, hipLaunchKernelGGL(k_dot<double>, g, kBlock, 0, s, (const double*)x, (const double*)y, n, partials),
                hipLaunchKernelGGL(k_dot<float>, g, kBlock, 0, s, (const float*)x, (const float*)y, n, partials));
  int rc = check_launch("dot");
  if (rc) return rc;
  return reduce_partials(partials, (int)g, out, s);
}
int vec_dot_zf(const double* x, const float* z, int64_t n, double* partials, double* out, hipStream_t s) {
  const unsigned g = dot_grid(n);
  hipLaunchKernelGGL(k_dot_zf, g, kBlock, 0, s, x, z, n, partials);
  int rc = check_launch("dot_zf");
  if (rc) return rc;
  return reduce_partials(partials, (int)g, out, s);
}
int cg_update_p_zf(double* p, const float* z, const double* num, const double* den, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p_zf, grid_for(n), kBlock, 0, s, p, z, num, den, n);
  return check_launch("cg_p_zf");
}
int cg_update_xr(double* x, double* r, const double* p, const double* v, const double* num,
                 const double* den, int64_t n, double* partials, hipStream_t s, double* save, float* r32) {
  const unsigned g = dot_grid(n);
  hipLaunchKernelGGL(k_cg_xr, g, kBlock, 0, s, x, r, p, v, num, den, n, partials, save, r32);
  int rc = check_launch("cg_xr");
  if (rc) return rc;
  return (int)g;  // caller reduces g partials
}
int cg_update_p(double* p, const double* z, const double* num, const double* den, int64_t n,
                hipStream_t s, bool negate) {
  hipLaunchKernelGGL(k_cg_p, grid_for(n), kBlock, 0, s, p, z, num, den, n, negate ? 1 : 0);
  return check_launch("cg_p");
}
// ------------------------------------------------------------------ several vectors
// Vector r of a block starts r * ld values after the first; blockIdx.y = r.
// Per-vector scalars are arrays indexed by r; active[r] == 0 freezes vector r
// (a converged solve of a batch).
static unsigned grid_for_b(int64_t n) {
  unsigned g = grid_for(n, 8);
  return g > (unsigned)kPartialsB ? (unsigned)kPartialsB : g;
}
template <typename A, typename B>
__global__ void k_convert_b(const A* x, int64_t ldx, B* y, int64_t ldy, int64_t n) {
  const A* xr = x + blockIdx.y * ldx;
  B* yr = y + blockIdx.y * ldy;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    yr[i] = (B)xr[i];
}
template <typename T>
__global__ void k_mul3_b(T a, const T* d, const T* b, T* z, int64_t n, int64_t ld) {
  const T* br = b + blockIdx.y * ld;
  T* zr = z + blockIdx.y * ld;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    zr[i] = a * d[i] * br[i];
}
// partials[r * gridDim.x + block] of x_r . y_r
__global__ void k_dot_b(const double* x, const double* y, int64_t n, int64_t ld, double* partials) {
  const double* xr = x + blockIdx.y * ld;
  const double* yr = y + blockIdx.y * ld;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += xr[i] * yr[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
}
// out[r] = sum of partials[r * np .. r * np + np), one block per vector
__global__ void k_reduce_b(const double* partials, int np, double* out) {
  const double* pr = partials + (int64_t)blockIdx.x * np;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += pr[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}
int reduce_strided(const double* partials, int64_t n, int nrhs, double* out, double* tmp, hipStream_t s) {
  if (nrhs < 1) return HMG_OK;
  const int64_t want = (n + kBlock - 1) / kBlock;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, kPartialsB));
  hipLaunchKernelGGL(k_reduce_strided, dim3(g, nrhs), kBlock, 0, s, partials, n, nrhs, tmp);
  TRY(check_launch("reduce_strided"));
  hipLaunchKernelGGL(k_reduce_b, nrhs, 1024, 0, s, (const double*)tmp, (int)g, out);
  return check_launch("reduce_b");
}
// omega_r = num[r] / den[r]; x_r += omega_r p_r; r_r -= omega_r v_r; partials of r_r . r_r;
// save[r] = num[r]; r32 (may be NULL): r_r rounded to FP32, vector r at r * ld32
// (the next V-cycle's right-hand side block)
// x = NULL: the step x += omega p is left to the next direction update
// (k_cg_p_zf_b) or k_cg_x_step, and omega is stored in alpha[q] instead.
__global__ void k_cg_xr_b(double* x, double* r, const double* p, const double* v, const double* num,
                          const double* den, int64_t n, int64_t ld, double* partials, double* save,
                          const int* active, float* r32, int64_t ld32, double* alpha) {
  const int q = blockIdx.y;
  const int64_t o = q * ld;
  float* const r32q = r32 ? r32 + q * ld32 : nullptr;
  double acc = 0.0;
  if (active[q]) {
    const double omega = num[q] / den[q];
    if (!x && blockIdx.x == 0 && threadIdx.x == 0) alpha[q] = omega;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      if (x) x[o + i] += omega * p[o + i];
      const double ri = r[o + i] - omega * v[o + i];
      r[o + i] = ri;
      if (r32q) r32q[i] = (float)ri;
      acc += ri * ri;
    }
  } else {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const double ri = r[o + i];
      if (r32q) r32q[i] = (float)ri;
      acc += ri * ri;
    }
  }
  double s = block_reduce(acc);
  if (threadIdx.x == 0) {
    partials[q * gridDim.x + blockIdx.x] = s;
    if (blockIdx.x == 0 && save && active[q]) save[q] = num[q];
  }
}
// partials[r * gridDim.x + block] of x_r . z_r with z in FP32 (vector r of z
// at r * ldz): the FP64 products of the FP32 preconditioned residual,
// widened exactly, without an FP64 copy of it
__global__ void k_dot_zf_b(const double* x, const float* z, int64_t n, int64_t ld, int64_t ldz, double* partials) {
  const double* xr = x + blockIdx.y * ld;
  const float* zr = z + blockIdx.y * ldz;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += xr[i] * (double)zr[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = s;
}
// p_r = z_r + beta_r p_r with z in FP32 (vector r at r * ldz), beta_r =
// num[r] / den[r]; den = NULL: p_r = z_r (the first direction).  x != NULL:
// first the previous iteration's step x_r += alpha[r] p_r (deferred by
// k_cg_xr_b), with the same p_r values.
__global__ void k_cg_p_zf_b(double* p, const float* z, const double* num, const double* den, int64_t n,
                            int64_t ld, int64_t ldz, const int* active, double* x, const double* alpha) {
  const int q = blockIdx.y;
  if (den && !active[q]) return;  // the first direction is set for every vector
  const double beta = den ? num[q] / den[q] : 0.0;
  double* const pq = p + q * ld;
  const float* const zq = z + q * ldz;
  if (x) {
    const double a = alpha[q];
    double* const xq = x + q * ld;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const double pi = pq[i];
      xq[i] += a * pi;
      pq[i] = den ? (double)zq[i] + beta * pi : (double)zq[i];
    }
    return;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    pq[i] = den ? (double)zq[i] + beta * pq[i] : (double)zq[i];
}
// x_r += alpha[r] p_r for the vectors r in mask (their deferred last step)
__global__ void k_cg_x_step(double* x, const double* p, const double* alpha, int64_t n, int64_t ld, uint64_t mask) {
  const int q = blockIdx.y;
  if (!((mask >> q) & 1)) return;
  const double a = alpha[q];
  double* const xq = x + q * ld;
  const double* const pq = p + q * ld;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    xq[i] += a * pq[i];
}
// p_r = z_r + beta_r p_r, beta_r = (+-) num[r] / den[r]
__global__ void k_cg_p_b(double* p, const double* z, const double* num, const double* den, int64_t n, int64_t ld,
                         int neg, const int* active) {
  const int q = blockIdx.y;
  if (!active[q]) return;
  const double beta = (neg ? -num[q] : num[q]) / den[q];
  const int64_t o = q * ld;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[o + i] = z[o + i] + beta * p[o + i];
}

int vec_convert_b(int from, const void* x, int64_t ldx, int to, void* y, int64_t ldy, int64_t n, int nrhs,
                  hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return HMG_OK;
  const dim3 g(grid_for(n), nrhs);
  if (from == HMG_F64 && to == HMG_F64)
    hipLaunchKernelGGL((k_convert_b<double, double>), g, kBlock, 0, s, (const double*)x, ldx, (double*)y, ldy, n);
  else if (from == HMG_F64)
    hipLaunchKernelGGL((k_convert_b<double, float>), g, kBlock, 0, s, (const double*)x, ldx, (float*)y, ldy, n);
  else if (to == HMG_F64)
    hipLaunchKernelGGL((k_convert_b<float, double>), g, kBlock, 0, s, (const float*)x, ldx, (double*)y, ldy, n);
  else
    hipLaunchKernelGGL((k_convert_b<float, float>), g, kBlock, 0, s, (const float*)x, ldx, (float*)y, ldy, n);
  return check_launch("convert_b");
}
int vec_mul3_b(int prec, double a, const void* d, const void* b, void* z, int64_t n, int64_t ld, int nrhs,
               hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return HMG_OK;
  const dim3 g(grid_for(n), nrhs);
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_mul3_b<double>, g, kBlock, 0, s, a, (const double*)d, (const double*)b,
                                   (double*)z, n, ld),
                hipLaunchKernelGGL(k_mul3_b<float>, g, kBlock, 0, s, (float)a, (const float*)d, (const float*)b,
                                   (float*)z, n, ld));
  return check_launch("mul3_b");
}
int vec_dot_b(const double* x, const double* y, int64_t n, int64_t ld, int nrhs, double* partials, double* out,
              hipStream_t s) {
  const unsigned g = grid_for_b(n);
  hipLaunchKernelGGL(k_dot_b, dim3(g, nrhs), kBlock, 0, s, x, y, n, ld, partials);
  TRY(check_launch("dot_b"));
  hipLaunchKernelGGL(k_reduce_b, nrhs, 1024, 0, s, (const double*)partials, (int)g, out);
  return check_launch("reduce_b");
}
int vec_dot_zf_b(const double* x, const float* z, int64_t n, int64_t ld, int64_t ldz, int nrhs, double* partials,
                 double* out, hipStream_t s) {
  const unsigned g = grid_for_b(n);
  hipLaunchKernelGGL(k_dot_zf_b, dim3(g, nrhs), kBlock, 0, s, x, z, n, ld, ldz, partials);
  TRY(check_launch("dot_zf_b"));
  hipLaunchKernelGGL(k_reduce_b, nrhs, 1024, 0, s, (const double*)partials, (int)g, out);
  return check_launch("reduce_b");
}
int cg_update_p_zf_b(double* p, const float* z, const double* num, const double* den, int64_t n, int64_t ld,
                     int64_t ldz, int nrhs, const int* active, hipStream_t s, double* x, const double* alpha) {
  hipLaunchKernelGGL(k_cg_p_zf_b, dim3(grid_for(n), nrhs), kBlock, 0, s, p, z, num, den, n, ld, ldz, active, x,
                     alpha);
  return check_launch("cg_p_zf_b");
}
int cg_step_x_b(double* x, const double* p, const double* alpha, int64_t n, int64_t ld, int nrhs, uint64_t mask,
                hipStream_t s) {
  if (!mask || nrhs < 1) return HMG_OK;
  hipLaunchKernelGGL(k_cg_x_step, dim3(grid_for(n), nrhs), kBlock, 0, s, x, p, alpha, n, ld, mask);
  return check_launch("cg_x_step");
}
int cg_update_xr_b(double* x, double* r, const double* p, const double* v, const double* num, const double* den,
                   int64_t n, int64_t ld, int nrhs, double* partials, double* rr, double* save, const int* active,
                   hipStream_t s, float* r32, int64_t ld32, double* alpha) {
  if (!x && !alpha) return fail(HMG_ERR_INVALID, "internal: deferred CG step without alpha");
  const unsigned g = grid_for_b(n);
  hipLaunchKernelGGL(k_cg_xr_b, dim3(g, nrhs), kBlock, 0, s, x, r, p, v, num, den, n, ld, partials, save, active,
                     r32, ld32, alpha);
  TRY(check_launch("cg_xr_b"));
  hipLaunchKernelGGL(k_reduce_b, nrhs, 1024, 0, s, (const double*)partials, (int)g, rr);
  return check_launch("reduce_b");
}
int cg_update_p_b(double* p, const double* z, const double* num, const double* den, int64_t n, int64_t ld, int nrhs,
                  const int* active, bool negate, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p_b, dim3(grid_for(n), nrhs), kBlock, 0, s, p, z, num, den, n, ld, negate ? 1 : 0, active);
  return check_launch("cg_p_b");
}

int vec_splitmix(int prec, uint64_t seed, void* x, int64_t n, hipStream_t s) {
  if (n <= 0) return HMG_OK;
  PREC_DISPATCH(prec, hipLaunchKernelGGL(k_splitmix<double>, grid_for(n), kBlock, 0, s, seed, (double*)x, n),
                hipLaunchKernelGGL(k_splitmix<float>, grid_for(n), kBlock, 0, s, seed, (float*)x, n));
  return check_launch("splitmix");
}

// ------------------------------------------------------------------ FE node sums
// Along one axis, node g lies in element q = g / k at local index g - q k;
// a node on an element boundary (local 0) is shared by q - 1 (local k) and q.
// Candidates are listed lower element first; `two` marks a shared node.
// Index arithmetic is 32-bit (node and DoF counts checked on the host).
struct Axis {
  int e0, l0, e1, l1;
  bool two;
};
__device__ __forceinline__ Axis node_axis(int g, int k, int Nd) {
  const int q = g / k, rem = g - q * k;
  Axis A;
  A.two = false;
  if (rem != 0) {
    A.e0 = q;
    A.l0 = rem;
  } else if (q == 0) {
    A.e0 = 0;
    A.l0 = 0;
  } else if (q == Nd) {
    A.e0 = Nd - 1;
    A.l0 = k;
  } else {
    A.e0 = q - 1;
    A.l0 = k;
    A.two = true;
  }
  A.e1 = A.two ? q : A.e0;
  A.l1 = A.two ? 0 : A.l0;
  return A;
}

struct FeGeo {
  int Nx, Ny, Nz, k, bcmask;
  int Mx, My, Mz;
  int64_t nnodes;
};
static FeGeo fe_geo(const Mesh& m, int k) {
  FeGeo g;
  g.Nx = m.N[0];
  g.Ny = m.N[1];
  g.Nz = m.N[2];
  g.k = k;
  g.bcmask = m.bcmask();
  g.Mx = m.N[0] * k + 1;
  g.My = m.N[1] * k + 1;
  g.Mz = m.N[2] * k + 1;
  g.nnodes = (int64_t)g.Mx * g.My * g.Mz;
  return g;
}
// (bitwise, without branches: it does not order the loads around it)
__device__ __forceinline__ bool node_fixed(const FeGeo& G, int gx, int gy, int gz) {
  const int m = G.bcmask;
  return ((gx == 0) & !(m & 1)) | ((gx == G.Mx - 1) & !(m & 2)) | ((gy == 0) & !(m & 4)) |
         ((gy == G.My - 1) & !(m & 8)) | ((gz == 0) & !(m & 16)) | ((gz == G.Mz - 1) & !(m & 32));
}

// Sum of a DG-layout vector over the elements sharing node (gx, gy, gz), in
// a fixed order (z, then y, then x candidates, lower first); *mult is the
// number of elements. The candidates' loads are all issued before the sum
// (each under its own condition), so they are in flight together; the sum
// then takes them in that order.
// K > 0: the degree at compile time (constant divisions); 0: G.k.
// NA more values (pointers also[a], NULL: none) are loaded after the
// candidates, in flight with them, into also_v[a].
template <typename T, int K = 0, int NA = 1>
__device__ __forceinline__ T node_gather_sum(const FeGeo& G, const T* dg, int gx, int gy, int gz, int* mult,
                                             const T* const (&also)[NA], T (&also_v)[NA]) {
  const int k = K ? K : G.k, n = k + 1, n3 = n * n * n;
  const Axis X = node_axis(gx, k, G.Nx), Y = node_axis(gy, k, G.Ny), Z = node_axis(gz, k, G.Nz);
  T v[8];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int ez = c ? Z.e1 : Z.e0, lz = c ? Z.l1 : Z.l0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int ey = b ? Y.e1 : Y.e0, ly = b ? Y.l1 : Y.l0;
      const int64_t row = (int64_t)G.Nx * (ey + G.Ny * ez);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ex = a ? X.e1 : X.e0, lx = a ? X.l1 : X.l0;
        const bool ok = (c == 0 || Z.two) && (b == 0 || Y.two) && (a == 0 || X.two);
        v[4 * c + 2 * b + a] = ok ? dg[(row + ex) * n3 + lx + n * (ly + n * lz)] : T(0);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < NA; ++a)
    if (also[a]) also_v[a] = *also[a];
  T s = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        if ((c == 0 || Z.two) && (b == 0 || Y.two) && (a == 0 || X.two)) s += v[4 * c + 2 * b + a];
  *mult = (1 + X.two) * (1 + Y.two) * (1 + Z.two);
  return s;
}

// Launch shape of the node kernels: x along gx (64 lanes), y along gy,
// z along gz; one node per thread.
constexpr int kNodeBx = 64, kNodeBy = 4;
static dim3 node_grid(const FeGeo& G) {
  return dim3((unsigned)((G.Mx + kNodeBx - 1) / kNodeBx), (unsigned)((G.My + kNodeBy - 1) / kNodeBy),
              (unsigned)G.Mz);
}

template <typename T, int MODE, int K>
__global__ void __launch_bounds__(kNodeBx * kNodeBy) k_fe_sum(FeGeo G, const T* dg, const T* u, T* out, const T* b,
                                                              const T* dinv, const T* xold, T sigma, T theta,
                                                              const int* skip, int nrhs, int64_t ld,
                                                              int64_t dgs) {
  if (skip && *skip) return;  // gated apply (iterative coarse solve)
  // grid z = node plane x vector, vector fastest: the vectors of one plane
  // run together and share the lines of dinv in L2
  const unsigned zr = blockIdx.z, uz = nrhs == 1 ? zr : zr / (unsigned)nrhs;
  const int gx = blockIdx.x * kNodeBx + threadIdx.x, gy = blockIdx.y * kNodeBy + threadIdx.y, gz = (int)uz;
  if (gx >= G.Mx || gy >= G.My) return;
  if (nrhs > 1) {  // vector r: its node vectors r * ld values on, its element-local results r * dgs
    const int64_t r = zr - uz * (unsigned)nrhs;
    u += r * ld;
    out += r * ld;
    if (MODE != OP_APPLY) b += r * ld;
    if (MODE == OP_CHEB && xold) xold += r * ld;
    dg += r * dgs;
  }
  const int64_t i = gx + (int64_t)G.Mx * (gy + (int64_t)G.My * gz);
  // the node-vector values are loaded with the gather (in flight together)
  const T* const ap[4] = {MODE == OP_CHEB ? u + i : nullptr, MODE == OP_CHEB && xold ? xold + i : nullptr,
                          MODE == OP_CHEB ? dinv + i : nullptr, MODE != OP_APPLY ? b + i : nullptr};
  T av[4] = {0, 0, 0, 0};  // x, x_old (NULL: 0), dinv, b
  int mult;
  T v = node_gather_sum<T, K, 4>(G, dg, gx, gy, gz, &mult, ap, av);
  const T x = av[0], xo = av[1], di = av[2], bi = av[3];
  if (node_fixed(G, gx, gy, gz)) v = MODE == OP_CHEB ? x : u[i];
  if (MODE == OP_APPLY) {
    out[i] = v;
  } else if (MODE == OP_RESID) {
    out[i] = bi - v;
  } else {
    out[i] = x + sigma * (x - xo) + theta * di * (bi - v);
  }
}
// fe (+)= free * w * E^T dg.  K > 0: the degree at compile time (constant
// divisions); 0: G.k.  Grid z = vector x node plane (vector slowest): vector
// r of fe starts r * ldf values on, of dg r * ldd values on.
template <typename T, int K>
__global__ void __launch_bounds__(kNodeBx * kNodeBy) k_c_sum(FeGeo G, const T* dg, T* fe, int weight_mult, int add,
                                                             int64_t ldd, int64_t ldf) {
  const unsigned r = blockIdx.z / (unsigned)G.Mz;
  const int gx = blockIdx.x * kNodeBx + threadIdx.x, gy = blockIdx.y * kNodeBy + threadIdx.y,
            gz = (int)(blockIdx.z - r * (unsigned)G.Mz);
  if (gx >= G.Mx || gy >= G.My) return;
  dg += r * ldd;
  fe += r * ldf;
  const int64_t i = gx + (int64_t)G.Mx * (gy + (int64_t)G.My * gz);
  const T* const ap[1] = {add ? fe + i : nullptr};
  T old[1] = {0};  // the value added to, in flight with the gather
  int mult;
  T v = node_gather_sum<T, K, 1>(G, dg, gx, gy, gz, &mult, ap, old);
  if (weight_mult) v /= (T)mult;
  if (node_fixed(G, gx, gy, gz)) v = 0;
  fe[i] = add ? old[0] + v : v;
}
// dg (+)= E (free * w * fe), one thread per DG value: grid x over the
// Nx n^3 values of one x-row of elements, y = ey, z = ez, so the element
// and local node come without run-time divisions (K > 0: the degree at
// compile time).  A node is shared along an axis when it is the element's
// first node and the element is not the first, or its last node and the
// element is not the last.  Grid z = vector x element plane (vector
// slowest): vector r of fe starts r * ldf values on, of dg r * ldd values on.
template <typename T, int K>
__global__ void __launch_bounds__(kBlock) k_c_inject(FeGeo G, const T* fe, T* dg, int weight_mult, int add,
                                                     int64_t ldd, int64_t ldf) {
  const int k = K ? K : G.k, n = k + 1, n2 = n * n, n3 = n2 * n;
  const int i = blockIdx.x * kBlock + threadIdx.x;  // value within the row
  if (i >= G.Nx * n3) return;
  const unsigned r = blockIdx.z / (unsigned)G.Nz;
  const int ey = blockIdx.y, ez = (int)(blockIdx.z - r * (unsigned)G.Nz);
  fe += r * ldf;
  dg += r * ldd;
  const int ex = i / n3, p = i - ex * n3;
  const int pz = p / n2, pr = p - pz * n2, py = pr / n, px = pr - py * n;
  const int gx = ex * k + px, gy = ey * k + py, gz = ez * k + pz;
  const int64_t o = (int64_t)(ez * G.Ny + ey) * G.Nx * n3 + i;
  const T old = add ? dg[o] : T(0);  // in flight with the node value
  T v = 0;
  if (!node_fixed(G, gx, gy, gz)) {
    v = fe[gx + (int64_t)G.Mx * (gy + (int64_t)G.My * gz)];
    if (weight_mult) {
      const int sx = (px == 0 && ex > 0) || (px == k && ex < G.Nx - 1);
      const int sy = (py == 0 && ey > 0) || (py == k && ey < G.Ny - 1);
      const int sz = (pz == 0 && ez > 0) || (pz == k && ez < G.Nz - 1);
      v /= (T)((1 + sx) * (1 + sy) * (1 + sz));
    }
  }
  dg[o] = add ? old + v : v;
}

template <typename T, int K>
static void launch_fe_sum(int mode, dim3 g, dim3 blk, const FeGeo& G, const T* dg, const void* u, void* out,
                          const void* b, const T* di, const void* xold, double sigma, double theta, hipStream_t s,
                          const int* skip, int nrhs, int64_t ld, int64_t dgs) {
  switch (mode) {
    case OP_RESID:
      hipLaunchKernelGGL((k_fe_sum<T, OP_RESID, K>), g, blk, 0, s, G, dg, (const T*)u, (T*)out,
                         (const T*)b, di, (const T*)xold, (T)sigma, (T)theta, skip, nrhs, ld, dgs);
      break;
    case OP_CHEB:
      hipLaunchKernelGGL((k_fe_sum<T, OP_CHEB, K>), g, blk, 0, s, G, dg, (const T*)u, (T*)out,
                         (const T*)b, di, (const T*)xold, (T)sigma, (T)theta, skip, nrhs, ld, dgs);
      break;
    default:
      hipLaunchKernelGGL((k_fe_sum<T, OP_APPLY, K>), g, blk, 0, s, G, dg, (const T*)u, (T*)out,
                         (const T*)b, di, (const T*)xold, (T)sigma, (T)theta, skip, nrhs, ld, dgs);
  }
}

template <typename T>
static int fe_sum_t(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                    const void* xold, double sigma, double theta, hipStream_t s, const int* skip,
                    const void* scratch, int nrhs, int64_t ld) {
  FeGeo G = fe_geo(L->mesh, L->k);
  if ((int64_t)G.Mz * nrhs > 65535) return fail(HMG_ERR_UNSUPPORTED, "FE level too large for the node grid");
  dim3 g = node_grid(G);
  g.z *= (unsigned)nrhs;
  const dim3 blk(kNodeBx, kNodeBy);
  const T* dg = (const T*)(scratch ? scratch : L->scratch());
  const T* di = (const T*)L->dinv();
  const int64_t dgs = L->n_dg;
#define HMG_FE_SUM(K) launch_fe_sum<T, K>(mode, g, blk, G, dg, u, out, b, di, xold, sigma, theta, s, skip, nrhs, ld, dgs)
  switch (G.k) {
    case 1: HMG_FE_SUM(1); break;
    case 2: HMG_FE_SUM(2); break;
    case 3: HMG_FE_SUM(3); break;
    case 4: HMG_FE_SUM(4); break;
    case 5: HMG_FE_SUM(5); break;
    case 6: HMG_FE_SUM(6); break;
    case 7: HMG_FE_SUM(7); break;
    default: HMG_FE_SUM(0);
  }
#undef HMG_FE_SUM
  return check_launch("fe_sum");
}
int fe_node_sum(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                const void* xold, double sigma, double theta, hipStream_t s, const int* skip,
                const void* scratch, int nrhs, int64_t ld) {
  if (nrhs < 1) return HMG_OK;
  if (L->prec == HMG_F64) return fe_sum_t<double>(L, mode, u, out, b, xold, sigma, theta, s, skip, scratch, nrhs, ld);
  return fe_sum_t<float>(L, mode, u, out, b, xold, sigma, theta, s, skip, scratch, nrhs, ld);
}

// ------------------------------------------------------------------ gated CG (coarse solve)
// Jacobi-preconditioned CG (Alg. 1 with D^{-1}) on one level; FP64 scalars
// in device memory; every kernel returns at once while *skip != 0, so a
// converged or unneeded solve costs launches only.
template <typename T>
__global__ void k_ccg_init(const T* b, const T* dinv, T* x, T* r, T* z, T* p, int64_t n, const int* skip) {
  if (*skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T bi = b[i], zi = dinv[i] * bi;
    x[i] = 0;
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
  }
}
template <typename T>
__global__ void k_ccg_xr(T* x, T* r, T* z, const T* p, const T* q, const T* dinv, int64_t n, const double* rz,
                         const double* pq, const int* skip) {
  if (*skip) return;
  // p.q = 0 only for p = 0 (b = 0, or a breakdown): no step, x stays
  const double pqv = *pq;
  const T a = pqv > 0 ? (T)(*rz / pqv) : T(0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const T ri = r[i] - a * q[i];
    r[i] = ri;
    z[i] = dinv[i] * ri;
  }
}
template <typename T>
__global__ void k_ccg_p(T* p, const T* z, int64_t n, const double* rzn, const double* rz, const int* skip) {
  if (*skip) return;
  const double rzv = *rz;
  const T beta = rzv != 0 ? (T)(*rzn / rzv) : T(0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}
__global__ void k_ccg_check(const double* rzn, const double* rz0, double tol2, int* skip, int* iters) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || *skip) return;
  *iters += 1;
  if (!(*rzn > tol2 * *rz0)) *skip = 1;  // converged, or NaN
}
template <typename T>
__global__ void k_dot_gated(const T* x, const T* y, int64_t n, double* partials, const int* skip) {
  if (*skip) return;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}
__global__ void k_reduce_gated(const double* partials, int np, double* out, const int* skip) {
  if (*skip) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partials[i];
  double s = block_reduce(acc);
  if (threadIdx.x == 0) *out = s;
}
__global__ void k_gate_to_skip(const double* gate, double accept2, int* skip, int* fallbacks, int* accepted) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double rr = gate[0], bb = gate[1];
  const bool ok = isfinite(rr) && rr <= accept2 * bb;
  *skip = ok ? 1 : 0;
  if (accepted) *accepted = ok ? 1 : 0;
  if (!ok) *fallbacks += 1;
}
__global__ void k_set_flag(int* flag, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = v;
}

int ccg_init(int prec, const void* b, const void* dinv, void* x, void* r, void* z, void* p, int64_t n,
             const int* skip, hipStream_t s) {
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_ccg_init<double>, grid_for(n), kBlock, 0, s, (const double*)b, (const double*)dinv,
                                   (double*)x, (double*)r, (double*)z, (double*)p, n, skip),
                hipLaunchKernelGGL(k_ccg_init<float>, grid_for(n), kBlock, 0, s, (const float*)b, (const float*)dinv,
                                   (float*)x, (float*)r, (float*)z, (float*)p, n, skip));
  return check_launch("ccg_init");
}
int ccg_xr(int prec, void* x, void* r, void* z, const void* p, const void* q, const void* dinv, int64_t n,
           const double* rz, const double* pq, const int* skip, hipStream_t s) {
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_ccg_xr<double>, grid_for(n), kBlock, 0, s, (double*)x, (double*)r, (double*)z,
                                   (const double*)p, (const double*)q, (const double*)dinv, n, rz, pq, skip),
                hipLaunchKernelGGL(k_ccg_xr<float>, grid_for(n), kBlock, 0, s, (float*)x, (float*)r, (float*)z,
                                   (const float*)p, (const float*)q, (const float*)dinv, n, rz, pq, skip));
  return check_launch("ccg_xr");
}
int ccg_p(int prec, void* p, const void* z, int64_t n, const double* rzn, const double* rz, const int* skip,
          hipStream_t s) {
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_ccg_p<double>, grid_for(n), kBlock, 0, s, (double*)p, (const double*)z, n, rzn, rz,
                                   skip),
                hipLaunchKernelGGL(k_ccg_p<float>, grid_for(n), kBlock, 0, s, (float*)p, (const float*)z, n, rzn, rz,
                                   skip));
  return check_launch("ccg_p");
}
int ccg_check(const double* rzn, const double* rz0, double tol2, int* skip, int* iters, hipStream_t s) {
  hipLaunchKernelGGL(k_ccg_check, 1, 64, 0, s, rzn, rz0, tol2, skip, iters);
  return check_launch("ccg_check");
}
int vec_dot_gated(int prec, const void* x, const void* y, int64_t n, double* partials, double* out,
                  const int* skip, hipStream_t s) {
  const unsigned g = dot_grid(n);
  PREC_DISPATCH(prec,
                hipLaunchKernelGGL(k_dot_gated<double>, g, kBlock, 0, s, (const double*)x, (const double*)y, n, partials,
                                   skip),
                hipLaunchKernelGGL(k_dot_gated<float>, g, kBlock, 0, s, (const float*)x, (const float*)y, n, partials,
                                   skip));
  hipLaunchKernelGGL(k_reduce_gated, 1, 1024, 0, s, (const double*)partials, (int)g, out, skip);
  return check_launch("dot_gated");
}
int gate_to_skip(const double* gate, double accept, int* skip, int* fallbacks, hipStream_t s, int* accepted) {
  hipLaunchKernelGGL(k_gate_to_skip, 1, 64, 0, s, gate, accept * accept, skip, fallbacks, accepted);
  return check_launch("gate_to_skip");
}
int set_flag(int* flag, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_flag, 1, 64, 0, s, flag, v);
  return check_launch("set_flag");
}

template <typename T, int K>
static void launch_c(bool inject, const FeGeo& G, const void* src, void* dst, int weight_mult, int add, int nv,
                     int64_t ldd, int64_t ldf, hipStream_t s) {
  if (inject) {
    const int n3 = (G.k + 1) * (G.k + 1) * (G.k + 1);
    const dim3 g((unsigned)((G.Nx * n3 + kBlock - 1) / kBlock), (unsigned)G.Ny, (unsigned)(G.Nz * nv));
    hipLaunchKernelGGL((k_c_inject<T, K>), g, dim3(kBlock), 0, s, G, (const T*)src, (T*)dst, weight_mult, add,
                       ldd, ldf);
  } else {
    dim3 g = node_grid(G);
    g.z *= (unsigned)nv;
    hipLaunchKernelGGL((k_c_sum<T, K>), g, dim3(kNodeBx, kNodeBy), 0, s, G, (const T*)src, (T*)dst, weight_mult,
                       add, ldd, ldf);
  }
}
template <typename T>
static void launch_c_k(bool inject, const FeGeo& G, const void* src, void* dst, int weight_mult, int add, int nv,
                       int64_t ldd, int64_t ldf, hipStream_t s) {
  switch (G.k) {
    case 1: launch_c<T, 1>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 2: launch_c<T, 2>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 3: launch_c<T, 3>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 4: launch_c<T, 4>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 5: launch_c<T, 5>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 6: launch_c<T, 6>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    case 7: launch_c<T, 7>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s); break;
    default: launch_c<T, 0>(inject, G, src, dst, weight_mult, add, nv, ldd, ldf, s);
  }
}
// The vectors go on grid z (planes x vectors): as many per launch as the
// 65535 limit of the grid allows.
template <typename T>
static void launch_c_v(bool inject, const FeGeo& G, const void* src, void* dst, int weight_mult, int add, int nrhs,
                       int64_t ldd, int64_t ldf, hipStream_t s) {
  const int64_t planes = inject ? G.Nz : G.Mz;
  const int per = (int)std::max<int64_t>(1, std::min<int64_t>(nrhs, 65535 / planes));
  const int64_t lds = inject ? ldf : ldd, ldt = inject ? ldd : ldf;  // source, destination strides
  for (int r = 0; r < nrhs; r += per)
    launch_c_k<T>(inject, G, (const T*)src + r * lds, (T*)dst + r * ldt, weight_mult, add, std::min(per, nrhs - r),
                  ldd, ldf, s);
}
int tr_c_inject(int prec, const Mesh& m, int k, const void* fe, void* dg, int weight_mult, int add,
                hipStream_t s, int nrhs, int64_t ld_fe, int64_t ld_dg) {
  FeGeo G = fe_geo(m, k);
  const int64_t n3 = (int64_t)(k + 1) * (k + 1) * (k + 1);
  if (nrhs < 1) return HMG_OK;
  if (m.n_el() * n3 >= (int64_t)1 << 31) return fail(HMG_ERR_UNSUPPORTED, "DG vector too long for the injection kernel");
  if (G.Ny > 65535 || G.Nz > 65535) return fail(HMG_ERR_UNSUPPORTED, "mesh too large for the injection grid");
  if (prec == HMG_F64) launch_c_v<double>(true, G, fe, dg, weight_mult, add, nrhs, ld_dg, ld_fe, s);
  else launch_c_v<float>(true, G, fe, dg, weight_mult, add, nrhs, ld_dg, ld_fe, s);
  return check_launch("c_inject");
}
int tr_c_sum(int prec, const Mesh& m, int k, const void* dg, void* fe, int weight_mult, int add,
             hipStream_t s, int nrhs, int64_t ld_dg, int64_t ld_fe) {
  FeGeo G = fe_geo(m, k);
  if (nrhs < 1) return HMG_OK;
  if (G.Mz > 65535) return fail(HMG_ERR_UNSUPPORTED, "FE level too large for the node grid");
  if (prec == HMG_F64) launch_c_v<double>(false, G, dg, fe, weight_mult, add, nrhs, ld_dg, ld_fe, s);
  else launch_c_v<float>(false, G, dg, fe, weight_mult, add, nrhs, ld_dg, ld_fe, s);
  return check_launch("c_sum");
}

// ------------------------------------------------------------------ DG p / h transfers
// Element-local tensor products with 1-D matrices P (nf x nc), P[i*nc + j]
// = coarse basis j at fine node i (Sec. 3.2: L2 projection = interpolation).
template <typename T>
struct TrArgs {
  T P[2][kMaxN * kMaxN];
  int nf, nc, kind;  // kind 0: p, 1: h
  int Nf[3];
  int64_t nel_f, nel_c;
  int W;  // output elements per wavefront
};

// Wavefront-local transfer kernel, sum-factorized: a wavefront stages W
// input elements in LDS and applies the 1-D matrix M (M = P_child for
// prolongation, P_child^T for restriction) direction by direction, one
// n-point line per lane and pass (lanes loop when a pass has more lines):
//   T1[o0, i1, i2] = sum_i0 M0[o0, i0] in[i0, i1, i2]
//   T2[o0, o1, i2] = sum_i1 M1[o1, i1] T1[o0, i1, i2]
//   out[o0, o1, o2] = sum_i2 M2[o2, i2] T2[o0, o1, i2]   (x fastest)
// W fills the LDS buffers (kTrBytes per buffer); the h-restriction adds the
// 8 children in a fixed order in registers (one output line per lane).  No
// workgroup barrier: four independent wavefronts per workgroup.  Grid y is
// the vector: vector r of in starts r * ldi values on, of out r * ldo.
constexpr int kTrBytes = 4096;  // bytes per LDS buffer and wavefront

__device__ __forceinline__ void tr_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NF, NC > 0: the node counts at compile time (unrolled 1-D products, the
// line arrays in registers); 0: taken from the arguments.
template <typename T, bool RESTRICT, int NF, int NC>
__global__ void __launch_bounds__(256) k_transfer(TrArgs<T> a, const T* in, T* out, int add, int64_t ldi,
                                                  int64_t ldo) {
  constexpr int BUF = kTrBytes / (int)sizeof(T);
  in += blockIdx.y * ldi;
  out += blockIdx.y * ldo;
  __shared__ T buf[4][2][BUF];
  __shared__ T Pl[4][2 * kMaxN * kMaxN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nf = NF ? NF : a.nf, nc = NC ? NC : a.nc;
  const int ni = RESTRICT ? nf : nc, no = RESTRICT ? nc : nf;
  const int ni2 = ni * ni, ni3 = ni2 * ni, no2 = no * no, no3 = no2 * no;
  const int W = a.W;
  const int64_t nel_out = RESTRICT ? a.nel_c : a.nel_f;
  const int64_t eb = ((int64_t)blockIdx.x * 4 + wave) * W;  // first output element of the wavefront
  T* const B = buf[wave][0];   // input elements, later T2
  T* const T1 = buf[wave][1];
  T* const P = Pl[wave];
  for (int i = lane; i < 2 * nf * nc; i += 64) {
    const int c = i / (nf * nc);
    P[i] = a.P[c][i - c * nf * nc];
  }
  const int Fx = a.Nf[0], Fy = a.Nf[1];
  const int Cx = Fx / 2, Cy = Fy / 2;
  const bool hres = RESTRICT && a.kind == 1;
  const int nchild = hres ? 8 : 1;
  // M_d(o, i) of child bit b: P[i][o] (restriction) or P[o][i] (prolongation)
  auto M = [&](int bit, int o, int i) -> T {
    const T* Pb = P + bit * nf * nc;
    return RESTRICT ? Pb[i * nc + o] : Pb[o * nc + i];
  };
  // child bit of direction d for output element le (h-transfers)
  auto bit = [&](int d, int c, int le) -> int {
    if (a.kind != 1) return 0;
    if (RESTRICT) return d == 0 ? (c & 1) : (d == 1 ? ((c >> 1) & 1) : (c >> 2));
    const int64_t eo = eb + le;
    if (eo >= nel_out) return 0;
    const unsigned u = (unsigned)eo, r = u / Fx, ez = r / Fy, ey = r - ez * Fy, ex = u - r * Fx;
    return d == 0 ? (ex & 1) : (d == 1 ? (ey & 1) : (ez & 1));
  };
  T acc[kMaxN];  // h-restriction: this lane's output line, summed over the children
#pragma unroll
  for (int j = 0; j < kMaxN; ++j) acc[j] = 0;
  // input element of output element eo (child c for the h-restriction)
  auto in_elem = [&](int64_t eo, int c) -> int64_t {
    if (a.kind != 1) return eo;
    const unsigned u = (unsigned)eo;
    if (RESTRICT) {  // coarse eo -> child c
      const unsigned r = u / Cx, cz = r / Cy, cy = r - cz * Cy, cx = u - r * Cx;
      return (2 * cx + (c & 1)) + (int64_t)Fx * ((2 * cy + ((c >> 1) & 1)) + (int64_t)Fy * (2 * cz + (c >> 2)));
    }
    // fine eo -> parent
    const unsigned r = u / Fx, ez = r / Fy, ey = r - ez * Fy, ex = u - r * Fx;
    return (ex >> 1) + (int64_t)Cx * ((ey >> 1) + (int64_t)Cy * (ez >> 1));
  };
  for (int c = 0; c < nchild; ++c) {
    tr_sync();
    if constexpr (NF > 0 && NC > 0) {
      // sizes at compile time: all of the lane's loads are issued before the
      // LDS stores, one memory round trip instead of one per value (values of
      // elements past the end are zeros whose results are not stored)
      constexpr int KL = BUF / 64;
      T v[KL];
#pragma unroll
      for (int j = 0; j < KL; ++j) {
        const int idx = lane + 64 * j;
        v[j] = T(0);
        if (idx < W * ni3) {
          const int le = idx / ni3, p = idx - le * ni3;
          const int64_t eo = eb + le;
          if (eo < nel_out) v[j] = in[in_elem(eo, c) * ni3 + p];
        }
      }
#pragma unroll
      for (int j = 0; j < KL; ++j)
        if (lane + 64 * j < W * ni3) B[lane + 64 * j] = v[j];
    } else {
      for (int idx = lane; idx < W * ni3; idx += 64) {
        const int le = idx / ni3, p = idx - le * ni3;
        const int64_t eo = eb + le;
        if (eo >= nel_out) continue;
        B[idx] = in[in_elem(eo, c) * ni3 + p];
      }
    }
    tr_sync();
    // pass 1, x-lines: (element le, line i1 + ni i2)
    for (int ln = lane; ln < W * ni2; ln += 64) {
      const int le = ln / ni2, line = ln - le * ni2;
      const int b0 = bit(0, c, le);
      T x[kMaxN];
      for (int i0 = 0; i0 < ni; ++i0) x[i0] = B[le * ni3 + ni * line + i0];
      for (int o0 = 0; o0 < no; ++o0) {
        T s = 0;
        for (int i0 = 0; i0 < ni; ++i0) s += M(b0, o0, i0) * x[i0];
        T1[le * no * ni2 + o0 + no * line] = s;
      }
    }
    tr_sync();
    // pass 2, y-lines: (element le, o0, i2); T2 overwrites the input
    for (int ln = lane; ln < W * no * ni; ln += 64) {
      const int le = ln / (no * ni), r = ln - le * (no * ni), o0 = r % no, i2 = r / no;
      const int b1 = bit(1, c, le);
      T x[kMaxN];
      for (int i1 = 0; i1 < ni; ++i1) x[i1] = T1[le * no * ni2 + o0 + no * (i1 + ni * i2)];
      for (int o1 = 0; o1 < no; ++o1) {
        T s = 0;
        for (int i1 = 0; i1 < ni; ++i1) s += M(b1, o1, i1) * x[i1];
        B[le * no2 * ni + o0 + no * (o1 + no * i2)] = s;
      }
    }
    tr_sync();
    // pass 3, z-lines: (element le, o0 + no o1)
    for (int ln = lane; ln < W * no2; ln += 64) {
      const int le = ln / no2, r = ln - le * no2;
      const int b2 = bit(2, c, le);
      T x[kMaxN];
      for (int i2 = 0; i2 < ni; ++i2) x[i2] = B[le * no2 * ni + r + no2 * i2];
      const int64_t eo = eb + le;
      for (int o2 = 0; o2 < no; ++o2) {
        T s = 0;
        for (int i2 = 0; i2 < ni; ++i2) s += M(b2, o2, i2) * x[i2];
        if (hres) {
          acc[o2] += s;  // one line per lane (W no^2 <= 64)
        } else if (eo < nel_out) {
          const int64_t g = eo * no3 + r + (int64_t)no2 * o2;
          out[g] = (!RESTRICT && add) ? out[g] + s : s;
        }
      }
    }
  }
  if (hres && lane < W * no2) {
    const int le = lane / no2, r = lane - le * no2;
    const int64_t eo = eb + le;
    if (eo < nel_out)
      for (int o2 = 0; o2 < no; ++o2) out[eo * no3 + r + (int64_t)no2 * o2] = acc[o2];
  }
}

template <typename T>
static TrArgs<T> tr_args(int kind, int nf, int nc, const int Nf[3], const double* P0, const double* P1,
                         bool restrict_) {
  TrArgs<T> a;
  {
    // W elements: the input, T1 and T2 of W elements fit the LDS buffers; the
    // h-restriction keeps one output line per lane (W no^2 <= 64)
    const int ni = restrict_ ? nf : nc, no = restrict_ ? nc : nf;
    const int buf = kTrBytes / (int)sizeof(T);
    const int per = std::max(ni * ni * ni, std::max(no * ni * ni, no * no * ni));
    int W = buf / per;
    if (restrict_ && kind == 1) W = std::min(W, 64 / (no * no));
    a.W = W < 1 ? 1 : W;
  }
  a.nf = nf;
  a.nc = nc;
  a.kind = kind;
  for (int d = 0; d < 3; ++d) a.Nf[d] = Nf[d];
  for (int i = 0; i < nf * nc; ++i) {
    a.P[0][i] = (T)P0[i];
    a.P[1][i] = (T)(P1 ? P1[i] : P0[i]);
  }
  a.nel_f = (int64_t)Nf[0] * Nf[1] * Nf[2];
  a.nel_c = kind == 1 ? a.nel_f / 8 : a.nel_f;
  return a;
}

// Launch with compile-time node counts for the (fine, coarse) pairs the
// hierarchies use (p: n -> n-1, n -> floor(k/2)+1, n -> 2; h and c: n -> n),
// the generic kernel otherwise.
template <typename T, bool R>
static void launch_transfer(int nf, int nc, unsigned g, const TrArgs<T>& a, const T* in, T* out, int add, int nrhs,
                            int64_t ldi, int64_t ldo, hipStream_t s) {
  const dim3 grid(g, (unsigned)nrhs);
#define HMG_TR(F, C)                                                                                    \
  if (nf == F && nc == C) {                                                                             \
    hipLaunchKernelGGL((k_transfer<T, R, F, C>), grid, 256, 0, s, a, in, out, add, ldi, ldo); \
    return;                                                                                             \
  }
  HMG_TR(2, 2) HMG_TR(3, 3) HMG_TR(4, 4) HMG_TR(5, 5) HMG_TR(6, 6) HMG_TR(7, 7) HMG_TR(8, 8)
  HMG_TR(3, 2) HMG_TR(4, 3) HMG_TR(5, 4) HMG_TR(6, 5) HMG_TR(7, 6) HMG_TR(8, 7)
  HMG_TR(4, 2) HMG_TR(5, 3) HMG_TR(6, 3) HMG_TR(7, 4) HMG_TR(8, 4)
  HMG_TR(5, 2) HMG_TR(6, 2) HMG_TR(7, 2) HMG_TR(8, 2)
#undef HMG_TR
  hipLaunchKernelGGL((k_transfer<T, R, 0, 0>), grid, 256, 0, s, a, in, out, add, ldi, ldo);
}

int tr_dg_prolongate(int prec, int kind, int nf, int nc, const int Nf[3], const double* P0,
                     const double* P1, const void* coarse, void* fine, int add, hipStream_t s, int nrhs,
                     int64_t ld_c, int64_t ld_f) {
  const int64_t nel_f = (int64_t)Nf[0] * Nf[1] * Nf[2];
  if (nel_f == 0 || nrhs < 1) return HMG_OK;
  if (nrhs > 65535) return fail(HMG_ERR_UNSUPPORTED, "too many vectors for one transfer launch");
  if (nel_f >= ((int64_t)1 << 31)) return fail(HMG_ERR_UNSUPPORTED, "too many elements for one transfer launch");
  if (prec == HMG_F64) {
    auto a = tr_args<double>(kind, nf, nc, Nf, P0, P1, false);
    const unsigned g = (unsigned)((nel_f + 4 * a.W - 1) / (4 * a.W));
    launch_transfer<double, false>(nf, nc, g, a, (const double*)coarse, (double*)fine, add, nrhs, ld_c, ld_f, s);
  } else {
    auto a = tr_args<float>(kind, nf, nc, Nf, P0, P1, false);
    const unsigned g = (unsigned)((nel_f + 4 * a.W - 1) / (4 * a.W));
    launch_transfer<float, false>(nf, nc, g, a, (const float*)coarse, (float*)fine, add, nrhs, ld_c, ld_f, s);
  }
  return check_launch("tr_prolong");
}
int tr_dg_restrict(int prec, int kind, int nf, int nc, const int Nf[3], const double* P0,
                   const double* P1, const void* fine, void* coarse, hipStream_t s, int nrhs, int64_t ld_f,
                   int64_t ld_c) {
  const int64_t nel_f = (int64_t)Nf[0] * Nf[1] * Nf[2];
  const int64_t nel_c = kind == 1 ? nel_f / 8 : nel_f;
  if (nel_c == 0 || nrhs < 1) return HMG_OK;
  if (nrhs > 65535) return fail(HMG_ERR_UNSUPPORTED, "too many vectors for one transfer launch");
  if (nel_f >= ((int64_t)1 << 31)) return fail(HMG_ERR_UNSUPPORTED, "too many elements for one transfer launch");
  if (prec == HMG_F64) {
    auto a = tr_args<double>(kind, nf, nc, Nf, P0, P1, true);
    const unsigned g = (unsigned)((nel_c + 4 * a.W - 1) / (4 * a.W));
    launch_transfer<double, true>(nf, nc, g, a, (const double*)fine, (double*)coarse, 0, nrhs, ld_f, ld_c, s);
  } else {
    auto a = tr_args<float>(kind, nf, nc, Nf, P0, P1, true);
    const unsigned g = (unsigned)((nel_c + 4 * a.W - 1) / (4 * a.W));
    launch_transfer<float, true>(nf, nc, g, a, (const float*)fine, (float*)coarse, 0, nrhs, ld_f, ld_c, s);
  }
  return check_launch("tr_restrict");
}

// ------------------------------------------------------------------ coarse solve
// x = Ainv b with the dense FP64 inverse of the coarsest operator; one
// wavefront per row, FP64 accumulation whatever the vector precision.
template <typename T>
__global__ void __launch_bounds__(256) k_coarse_gemv(const double* Ainv, const T* b, T* x, int n) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* Ar = Ainv + (int64_t)row * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += Ar[j] * (double)b[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[row] = (T)acc;
}
int coarse_gemv(int prec, const double* Ainv, const void* b, void* x, int n, hipStream_t s) {
  const unsigned g = (unsigned)((n + 3) / 4);
  PREC_DISPATCH(prec, hipLaunchKernelGGL(k_coarse_gemv<double>, g, 256, 0, s, Ainv, (const double*)b, (double*)x, n),
                hipLaunchKernelGGL(k_coarse_gemv<float>, g, 256, 0, s, Ainv, (const float*)b, (float*)x, n));
  return check_launch("coarse_gemv");
}

}  // namespace hmg
