// Matrix-free SIPG / continuous-FE Laplace operator for gfx950 (Sec. 4,
// eq:MatrixFreeAbstractNotation) and its launchers.
//
// Work decomposition: one workgroup owns E consecutive elements (x-fastest
// numbering), n^2 threads per element.  Thread t of an element owns one
// line of n points along a direction that changes from phase to phase
// (x-lines: t = j + n*l, y-lines: t = i + n*l, z-lines: t = i + n*j), so
// every 1-D contraction is a register-only loop with the n x n table in
// scalar registers (kernel arguments), and only the change of direction
// goes through LDS.
//
// Cell integral (Sec. 4): interpolate to Gauss points (3 sweeps with S),
// collocation gradient at the Gauss points (3 sweeps with D), quadrature-
// point operator (stored w|det J| J^{-1} J^{-T} for curved cells, constant
// diagonal for affine ones), integration with the transposed sweeps.
//
// Face integrals (cell-based loop, Sec. 2 fluxes): each element evaluates
// all six faces from its own side; the neighbour trace is gathered from
// global memory (L2).  Traces are formed on the nodal face (GLL: the face
// value is the end node, the normal derivative a dot product along the
// line), taken to the face Gauss points with 2-D sweeps, the flux is
// applied pointwise, and the test side returns to the nodal face with the
// transposed sweeps and is added to the element result.  No element writes
// to another element's output: deterministic, no atomics.
#include "hmg_internal.h"

namespace hmg {

#ifndef HMG_DISPATCH_ONLY
template <int N>
struct Cfg {
  static constexpr int NT = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int E = (256 / NT) >= 1 ? 256 / NT : 1;
  static constexpr int THREADS = ((E * NT + 63) / 64) * 64;
  static constexpr int FACE = 12 * NT;
  static constexpr int WORK = (2 * N3 > FACE) ? 2 * N3 : FACE;
  static constexpr int PER = N3 + WORK;
};

template <int N, typename T>
struct OpArgs {
  const T* u;
  T* out;
  const T* b;
  const T* dinv;
  const T* xold;
  T sigma, theta;
  double* partials;
  const T* metric;
  const T* face[3];
  const T* tau;
  int64_t nel;
  int Nx, Ny, Nz, bcmask;
  T h[3];
  OpTab<N, T> tab;
};

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of element batches so neighbouring elements share an L2.
__device__ __forceinline__ int xcd_block() {
  int nb = gridDim.x, x = blockIdx.x & 7, y = blockIdx.x >> 3;
  int per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + y;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  }
  return s;
}

// ------------------------------------------------------------------ faces
template <int N, typename T, bool CURVED, int d>
__device__ __forceinline__ void face_pass(const OpArgs<N, T>& a, const T* A, T* F, bool act, int t,
                                          int64_t e, const int ec[3], T vacc[N]) {
  constexpr int NT = N * N, N3 = N * N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  const auto& tb = a.tab;
  const int ta = t % N, tbb = t / N;
  auto lidx = [&](int m) -> int {
    if (d == 0) return m + N * t;
    if (d == 1) return ta + N * m + NT * tbb;
    return t + NT * m;
  };
  const int Nd = d == 0 ? a.Nx : (d == 1 ? a.Ny : a.Nz);
  const int64_t stride = d == 0 ? 1 : (d == 1 ? (int64_t)a.Nx : (int64_t)a.Nx * a.Ny);
  T Po[2] = {0, 0}, Qo[2] = {0, 0}, Pn[2] = {0, 0}, Qn[2] = {0, 0};
  bool has[2] = {false, false};
  T taue = 0, taun[2] = {0, 0};
  if (act) {
    T line[N];
#pragma unroll
    for (int m = 0; m < N; ++m) line[m] = A[lidx(m)];
    Po[0] = line[0];
    Po[1] = line[N - 1];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      Qo[0] += tb.dl0[m] * line[m];
      Qo[1] += tb.dl1[m] * line[m];
    }
    taue = a.tau[e];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      has[s] = s ? (ec[d] + 1 < Nd) : (ec[d] > 0);
      if (has[s]) {
        const int64_t en = e + (s ? stride : -stride);
        const T* un = a.u + en * N3;
        T nl[N];
#pragma unroll
        for (int m = 0; m < N; ++m) nl[m] = un[lidx(m)];
        Pn[s] = s ? nl[0] : nl[N - 1];
        T q = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) q += (s ? tb.dl0[m] : tb.dl1[m]) * nl[m];
        Qn[s] = q;
        taun[s] = a.tau[en];
      }
    }
  }
  bool dir[2], neu[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool isneu = (a.bcmask >> (2 * d + s)) & 1;
    dir[s] = !has[s] && !isneu;
    neu[s] = !has[s] && isneu;
  }

  if constexpr (!CURVED) {
    // Affine: n^T J^{-T} = (2s-1)/h_d e_d on both sides, surface weight
    // h_a h_b w_a w_b, so the flux collapses to two nodal face arrays
    // R1 = tau [u] - c {Q}/... followed by the face mass matrix M x M.
    const T hd = a.h[d], hab = a.h[da] * a.h[db];
    T R[4];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T cd = s ? T(1) / hd : T(-1) / hd;
      const T tauF = has[s] ? (taue > taun[s] ? taue : taun[s]) : taue;
      T Pj = has[s] ? Po[s] - Pn[s] : (dir[s] ? T(2) * Po[s] : T(0));
      T Qs = has[s] ? Qo[s] + Qn[s] : (dir[s] ? T(2) * Qo[s] : T(0));
      if (neu[s]) Pj = Qs = 0;
      R[2 * s] = tauF * Pj - T(0.5) * cd * Qs;
      R[2 * s + 1] = -T(0.5) * cd * Pj;
    }
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c) F[c * NT + t] = R[c];
    __syncthreads();
    T Z[4] = {0, 0, 0, 0};
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < N; ++q) Z[c] += tb.M[ta * N + q] * F[c * NT + q + N * tbb];
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c) F[c * NT + t] = Z[c];
    __syncthreads();
    T W[4] = {0, 0, 0, 0};
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int q = 0; q < N; ++q) W[c] += tb.M[tbb * N + q] * F[c * NT + ta + N * q];
        W[c] *= hab;
      }
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c) F[c * NT + t] = W[c];
    __syncthreads();
  } else {
    // Curved: full reference gradients of both traces at the face Gauss
    // points, n^T J^{-T} of both sides and the surface weight per point.
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        F[(s * 6 + 0) * NT + t] = Po[s];
        F[(s * 6 + 1) * NT + t] = Qo[s];
        F[(s * 6 + 2) * NT + t] = Pn[s];
        F[(s * 6 + 3) * NT + t] = Qn[s];
      }
    __syncthreads();
    T X[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) X[c] = 0;
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = tb.S[ta * N + q], sp = tb.Sp[ta * N + q];
          const T po = F[(s * 6 + 0) * NT + q + N * tbb], qo = F[(s * 6 + 1) * NT + q + N * tbb];
          const T pn = F[(s * 6 + 2) * NT + q + N * tbb], qn = F[(s * 6 + 3) * NT + q + N * tbb];
          X[s * 6 + 0] += sv * po;
          X[s * 6 + 1] += sp * po;
          X[s * 6 + 2] += sv * qo;
          X[s * 6 + 3] += sv * pn;
          X[s * 6 + 4] += sp * pn;
          X[s * 6 + 5] += sv * qn;
        }
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 12; ++c) F[c * NT + t] = X[c];
    __syncthreads();
    T Tt[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Tt[c] = 0;
    if (act) {
      const int pos_base = ec[d];
      const int ea = ec[da], eb = ec[db];
      const int Na = da == 0 ? a.Nx : a.Ny;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        T uo = 0, ao = 0, bo = 0, dd = 0, un = 0, an = 0, bn = 0, dn = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = tb.S[tbb * N + q], sp = tb.Sp[tbb * N + q];
          const int o = ta + N * q;
          const T x0 = F[(s * 6 + 0) * NT + o], x1 = F[(s * 6 + 1) * NT + o],
                  x2 = F[(s * 6 + 2) * NT + o];
          const T x3 = F[(s * 6 + 3) * NT + o], x4 = F[(s * 6 + 4) * NT + o],
                  x5 = F[(s * 6 + 5) * NT + o];
          uo += sv * x0;
          ao += sv * x1;
          bo += sp * x0;
          dd += sv * x2;
          un += sv * x3;
          an += sv * x4;
          bn += sp * x3;
          dn += sv * x5;
        }
        if (neu[s]) continue;
        const int64_t f = (pos_base + s) + (int64_t)(Nd + 1) * (ea + (int64_t)Na * eb);
        const T* g = a.face[d] + f * 7 * NT;
        T cL[3], cR[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          cL[r] = g[r * NT + t];
          cR[r] = g[(3 + r) * NT + t];
        }
        const T dA = g[6 * NT + t];
        T co[3], cn[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          co[r] = s ? cL[r] : -cR[r];
          cn[r] = s ? cR[r] : -cL[r];
        }
        const T dno = co[d] * dd + co[da] * ao + co[db] * bo;
        T jump, avg, tauF;
        if (has[s]) {
          const T dnn = cn[d] * dn + cn[da] * an + cn[db] * bn;
          jump = uo - un;
          avg = T(0.5) * (dno + dnn);
          tauF = taue > taun[s] ? taue : taun[s];
        } else {
          jump = T(2) * uo;
          avg = dno;
          tauF = taue;
        }
        const T vt = (tauF * jump - avg) * dA;
        const T gt = T(-0.5) * jump * dA;
        Tt[s * 4 + 0] = vt;
        Tt[s * 4 + 1] = gt * co[da];
        Tt[s * 4 + 2] = gt * co[db];
        Tt[s * 4 + 3] = gt * co[d];
      }
    }
    __syncthreads();
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) F[(s * 6 + c) * NT + t] = Tt[s * 4 + c];
    __syncthreads();
    T Y[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) Y[c] = 0;
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = tb.S[q * N + tbb], sp = tb.Sp[q * N + tbb];
          const int o = ta + N * q;
          Y[s * 3 + 0] += sv * F[(s * 6 + 0) * NT + o] + sp * F[(s * 6 + 2) * NT + o];
          Y[s * 3 + 1] += sv * F[(s * 6 + 1) * NT + o];
          Y[s * 3 + 2] += sv * F[(s * 6 + 3) * NT + o];
        }
    __syncthreads();
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) F[(s * 6 + c) * NT + t] = Y[s * 3 + c];
    __syncthreads();
    T Pq[4] = {0, 0, 0, 0};
    if (act)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = tb.S[q * N + ta], sp = tb.Sp[q * N + ta];
          const int o = q + N * tbb;
          Pq[s * 2 + 0] += sv * F[(s * 6 + 0) * NT + o] + sp * F[(s * 6 + 1) * NT + o];
          Pq[s * 2 + 1] += sv * F[(s * 6 + 2) * NT + o];
        }
    __syncthreads();
    if (act)
#pragma unroll
      for (int c = 0; c < 4; ++c) F[c * NT + t] = Pq[c];
    __syncthreads();
  }
  // F[(2s)*NT + node] = plane contribution, F[(2s+1)*NT + node] = weight of
  // l_p'(s) along the face normal.  Add into this thread's x-line.
  if (act) {
    const int j = t % N, l = t / N;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* Pv = F + (2 * s) * NT;
      const T* Qv = F + (2 * s + 1) * NT;
      const int endp = s * (N - 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T dli = s ? tb.dl1[i] : tb.dl0[i];
        if (d == 0) {
          vacc[i] += (i == endp ? Pv[t] : T(0)) + dli * Qv[t];
        } else if (d == 1) {
          const T dlj = s ? tb.dl1[j] : tb.dl0[j];
          vacc[i] += (j == endp ? Pv[i + N * l] : T(0)) + dlj * Qv[i + N * l];
        } else {
          const T dll = s ? tb.dl1[l] : tb.dl0[l];
          vacc[i] += (l == endp ? Pv[i + N * j] : T(0)) + dll * Qv[i + N * j];
        }
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ operator
template <int N, typename T, bool CURVED, bool FE, int MODE>
__global__ void __launch_bounds__(Cfg<N>::THREADS) op_kernel(const OpArgs<N, T> a) {
  using C = Cfg<N>;
  constexpr int NT = C::NT, N3 = C::N3, E = C::E, PER = C::PER;
  __shared__ T smem[E * PER];
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const int le = tid / NT, t = tid - le * NT;
  const int64_t e0 = (int64_t)xcd_block() * E;
  const int64_t e = e0 + le;
  const bool act = (le < E) && (e < a.nel);
  T* A = smem + (le < E ? le : 0) * PER;
  T* B = A + N3;
  T* Cc = B + N3;
  const auto& tb = a.tab;
  int ec[3] = {0, 0, 0};
  if (act) {
    ec[0] = (int)(e % a.Nx);
    const int64_t r = e / a.Nx;
    ec[1] = (int)(r % a.Ny);
    ec[2] = (int)(r / a.Ny);
  }
  const int64_t nloc = a.nel - e0 < E ? a.nel - e0 : E;
  const int nload = (int)nloc * N3;

  // ---- gather the block's elements into LDS (coalesced)
  if constexpr (!FE) {
    const T* src = a.u + e0 * N3;
    for (int idx = tid; idx < nload; idx += C::THREADS) {
      const int li = idx / N3;
      smem[li * PER + (idx - li * N3)] = src[idx];
    }
  } else {
    constexpr int k = N - 1;
    const int64_t Mx = (int64_t)a.Nx * k + 1, My = (int64_t)a.Ny * k + 1, Mz = (int64_t)a.Nz * k + 1;
    for (int idx = tid; idx < nload; idx += C::THREADS) {
      const int li = idx / N3, p = idx - li * N3;
      const int64_t ee = e0 + li;
      const int64_t gx = (ee % a.Nx) * k + p % N;
      const int64_t rr = ee / a.Nx;
      const int64_t gy = (rr % a.Ny) * k + (p / N) % N;
      const int64_t gz = (rr / a.Ny) * k + p / NT;
      const int m = a.bcmask;
      const bool fixed = (gx == 0 && !(m & 1)) || (gx == Mx - 1 && !(m & 2)) ||
                         (gy == 0 && !(m & 4)) || (gy == My - 1 && !(m & 8)) ||
                         (gz == 0 && !(m & 16)) || (gz == Mz - 1 && !(m & 32));
      smem[li * PER + p] = fixed ? T(0) : a.u[gx + Mx * (gy + My * gz)];
    }
  }
  __syncthreads();

  T vacc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) vacc[i] = 0;
  if constexpr (!FE) {
    face_pass<N, T, CURVED, 0>(a, A, B, act, t, e, ec, vacc);
    face_pass<N, T, CURVED, 1>(a, A, B, act, t, e, ec, vacc);
    face_pass<N, T, CURVED, 2>(a, A, B, act, t, e, ec, vacc);
  }

  const int ta = t % N, tbb = t / N;
  // ---- cell: interpolation to Gauss points, x then y then z
  if (act) {
    T in[N], o[N];
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = A[m + N * t];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.S[q * N + m] * in[m];
      o[q] = s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) A[q + N * t] = o[q];
  }
  __syncthreads();
  if (act) {
    T in[N], o[N];
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = A[ta + N * m + NT * tbb];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.S[q * N + m] * in[m];
      o[q] = s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) A[ta + N * q + NT * tbb] = o[q];
  }
  __syncthreads();
  T gz[N];
  if (act) {
    T in[N], uq[N];
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = A[t + NT * m];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.S[q * N + m] * in[m];
      uq[q] = s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.D[q * N + m] * uq[m];
      gz[q] = s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) A[t + NT * q] = uq[q];
  }
  __syncthreads();
  // ---- collocation derivatives in x (into B) and y (into C)
  if (act) {
    T in[N];
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = A[m + N * t];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.D[q * N + m] * in[m];
      B[q + N * t] = s;
    }
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = A[ta + N * m + NT * tbb];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += tb.D[q * N + m] * in[m];
      Cc[ta + N * q + NT * tbb] = s;
    }
  }
  __syncthreads();
  // ---- quadrature-point operator on z-lines, start of integration in z
  if (act) {
    T fx[N], fy[N], fz[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T gx = B[t + NT * m], gy = Cc[t + NT * m], g3 = gz[m];
      if constexpr (CURVED) {
        const T* G = a.metric + e * 6 * N3 + t + NT * m;
        const T g00 = G[0], g11 = G[N3], g22 = G[2 * N3], g01 = G[3 * N3], g02 = G[4 * N3],
                g12 = G[5 * N3];
        fx[m] = g00 * gx + g01 * gy + g02 * g3;
        fy[m] = g01 * gx + g11 * gy + g12 * g3;
        fz[m] = g02 * gx + g12 * gy + g22 * g3;
      } else {
        const T w = tb.w[ta] * tb.w[tbb] * tb.w[m];
        fx[m] = w * (a.h[1] * a.h[2] / a.h[0]) * gx;
        fy[m] = w * (a.h[0] * a.h[2] / a.h[1]) * gy;
        fz[m] = w * (a.h[0] * a.h[1] / a.h[2]) * g3;
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        s1 += tb.S[q * N + i] * fx[q];
        s2 += tb.S[q * N + i] * fy[q];
        s3 += tb.Sp[q * N + i] * fz[q];
      }
      B[t + NT * i] = s1;
      Cc[t + NT * i] = s2;
      A[t + NT * i] = s3;
    }
  }
  __syncthreads();
  // ---- integration in y
  if (act) {
    T cz[N], az[N], bz[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int o = ta + N * m + NT * tbb;
      cz[m] = A[o];
      az[m] = B[o];
      bz[m] = Cc[o];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s1 = 0, s2 = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        s1 += tb.S[q * N + i] * cz[q] + tb.Sp[q * N + i] * bz[q];
        s2 += tb.S[q * N + i] * az[q];
      }
      const int o = ta + N * i + NT * tbb;
      A[o] = s1;
      B[o] = s2;
    }
  }
  __syncthreads();
  // ---- integration in x, add the face terms, stage for the store
  if (act) {
    T dy[N], ey[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      dy[m] = A[m + N * t];
      ey[m] = B[m + N * t];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T s = vacc[i];
#pragma unroll
      for (int q = 0; q < N; ++q) s += tb.S[q * N + i] * dy[q] + tb.Sp[q * N + i] * ey[q];
      A[i + N * t] = s;
    }
  }
  __syncthreads();

  // ---- coalesced epilogue
  const int64_t gbase = e0 * N3;
  double acc = 0.0;
  for (int idx = tid; idx < nload; idx += C::THREADS) {
    const int li = idx / N3;
    const T val = smem[li * PER + (idx - li * N3)];
    const int64_t g = gbase + idx;
    if constexpr (FE || MODE == OP_APPLY) {
      a.out[g] = val;
    } else if constexpr (MODE == OP_RESID) {
      a.out[g] = a.b[g] - val;
    } else if constexpr (MODE == OP_CHEB) {
      const T x = a.u[g];
      a.out[g] = x + a.sigma * (x - a.xold[g]) + a.theta * a.dinv[g] * (a.b[g] - val);
    } else {
      a.out[g] = val;
      acc += (double)a.u[g] * (double)val;
    }
  }
  if constexpr (!FE && MODE == OP_DOT) {
    const double s = block_sum(acc, red);
    if (tid == 0) a.partials[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ launchers
template <int N, typename T>
static OpArgs<N, T> make_args(const hmg_level* L) {
  OpArgs<N, T> a;
  a.u = nullptr;
  a.out = nullptr;
  a.b = nullptr;
  a.dinv = (const T*)L->dinv();
  a.xold = nullptr;
  a.sigma = a.theta = 0;
  a.partials = L->partials();
  a.metric = (const T*)L->metric();
  for (int d = 0; d < 3; ++d) a.face[d] = (const T*)L->face(d);
  a.tau = (const T*)L->tau();
  a.nel = L->n_el;
  a.Nx = L->mesh.N[0];
  a.Ny = L->mesh.N[1];
  a.Nz = L->mesh.N[2];
  a.bcmask = L->mesh.bcmask();
  for (int d = 0; d < 3; ++d) a.h[d] = (T)L->mesh.h(d);
  a.tab = make_tab<N, T>(L->basis);
  return a;
}

template <int N, typename T, bool CURVED, bool FE>
static int run_op(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                  const void* xold, double sigma, double theta, int* nparts, hipStream_t s) {
  using C = Cfg<N>;
  OpArgs<N, T> a = make_args<N, T>(L);
  a.u = (const T*)u;
  a.out = (T*)(FE ? L->scratch() : out);
  a.b = (const T*)b;
  a.xold = (const T*)xold;
  a.sigma = (T)sigma;
  a.theta = (T)theta;
  const int64_t nb = (L->n_el + C::E - 1) / C::E;
  if (nb > INT32_MAX) return fail(HMG_ERR_UNSUPPORTED, "mesh too large for one launch");
  if (nparts) *nparts = (int)nb;
  dim3 grid((unsigned)nb), block(C::THREADS);
  if (FE) {
    hipLaunchKernelGGL((op_kernel<N, T, CURVED, true, OP_APPLY>), grid, block, 0, s, a);
  } else {
    switch (mode) {
      case OP_APPLY:
        hipLaunchKernelGGL((op_kernel<N, T, CURVED, false, OP_APPLY>), grid, block, 0, s, a);
        break;
      case OP_RESID:
        hipLaunchKernelGGL((op_kernel<N, T, CURVED, false, OP_RESID>), grid, block, 0, s, a);
        break;
      case OP_CHEB:
        hipLaunchKernelGGL((op_kernel<N, T, CURVED, false, OP_CHEB>), grid, block, 0, s, a);
        break;
      default:
        hipLaunchKernelGGL((op_kernel<N, T, CURVED, false, OP_DOT>), grid, block, 0, s, a);
        break;
    }
  }
  int rc = check_launch("op_kernel");
  if (rc) return rc;
  if (FE) return fe_node_sum(L, mode, u, out, b, xold, sigma, theta, s);
  return HMG_OK;
}

template <int N, typename T>
static int dispatch_op(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                       const void* xold, double sigma, double theta, int* nparts, hipStream_t s) {
  const bool curved = L->mesh.curved, fe = L->space == HMG_FE;
  if (curved) {
    if (fe) return run_op<N, T, true, true>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
    return run_op<N, T, true, false>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
  }
  if (fe) return run_op<N, T, false, true>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
  return run_op<N, T, false, false>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
}

#define HMG_CAT2(a, b) a##b
#define HMG_CAT(a, b) HMG_CAT2(a, b)
#ifdef HMG_ONLY_N
int HMG_CAT(op_launch_n, HMG_ONLY_N)(const hmg_level* L, int mode, const void* u, void* out,
                                      const void* b, const void* xold, double sigma, double theta,
                                      int* nparts, hipStream_t s) {
  if (L->prec == HMG_F64)
    return dispatch_op<HMG_ONLY_N, double>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
  return dispatch_op<HMG_ONLY_N, float>(L, mode, u, out, b, xold, sigma, theta, nparts, s);
}
#endif
#endif  // HMG_DISPATCH_ONLY

#ifdef HMG_DISPATCH_ONLY
#define HMG_DECL(N)                                                                          \
  int op_launch_n##N(const hmg_level*, int, const void*, void*, const void*, const void*,    \
                     double, double, int*, hipStream_t);
HMG_DECL(2)
HMG_DECL(3)
HMG_DECL(4)
HMG_DECL(5)
HMG_DECL(6)
HMG_DECL(7)
HMG_DECL(8)

int launch_operator(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                    const void* xold, double sigma, double theta, int* nparts, hipStream_t s) {
  if (L->n_el == 0) return HMG_OK;
  switch (L->n) {
#define HMG_CASE(N) \
  case N: return op_launch_n##N(L, mode, u, out, b, xold, sigma, theta, nparts, s);
    HMG_CASE(2) HMG_CASE(3) HMG_CASE(4) HMG_CASE(5) HMG_CASE(6) HMG_CASE(7) HMG_CASE(8)
#undef HMG_CASE
  }
  return fail(HMG_ERR_UNSUPPORTED, "degree must be 1..7");
}

#endif  // HMG_DISPATCH_ONLY

}  // namespace hmg
