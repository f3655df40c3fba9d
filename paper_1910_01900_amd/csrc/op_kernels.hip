// Matrix-free SIPG / continuous-FE Laplace operator for gfx950 (Sec. 4,
// eq:MatrixFreeAbstractNotation) and its launchers.
//
// Work decomposition: every wavefront owns EW = 64 / n^2 elements outright
// (n^2 lanes per element) and a private LDS region; all exchanges between
// lanes stay inside the wavefront, so phases are separated by wavefront
// fences instead of workgroup barriers and the four wavefronts of a
// workgroup progress independently (the latency of one hides behind the
// others).  Lane t of an element owns one line of n points along the
// direction of the current phase (x-lines: t = j + n*l, y-lines:
// t = i + n*l, z-lines: t = i + n*j), so every 1-D contraction is a
// register-only loop with the n x n tables in scalar registers; LDS only
// changes the direction.
//
// Curvilinear cells (Sec. 4): interpolation to the Gauss points (3 sweeps
// with S), collocation gradient (3 sweeps with D), the stored metric
// w |det J| J^{-1} J^{-T}, integration (transposed sweeps).  Faces (Sec. 2
// fluxes, cell-based loop): the own trace and reference gradient at a face
// point are extrapolated along the normal line from the cell's Gauss-point
// values (Gauss Lagrange basis at 0 or 1; exact, both are polynomials of
// degree <= k along that line); the neighbour's trace comes from its nodal
// face data (global memory / L2) with 2-D face sweeps; the face test
// functions go back into the cell integration arrays along the same normal
// line, so the face integrals share the cell's integration sweeps.  Affine
// cells use the nodal form sum_d c_d K_d (x) M (x) M (7 sweeps) and their
// faces collapse to face mass-matrix products in nodal space.  No element
// writes another element's output: deterministic, no atomics.
#include "hmg_internal.h"

namespace hmg {

#ifndef HMG_DISPATCH_ONLY
template <int N, bool CURVED, bool FE>
struct Cfg {
  static constexpr int NT = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int EW = 64 / NT >= 1 ? 64 / NT : 1;  // elements per wavefront
  static constexpr int WAVES = 4;
  static constexpr int EB = EW * WAVES;  // elements per workgroup
  // LDS values per element: curved uses 4 arrays (value/flux x, y, z) and,
  // for DG, 18 n^2 neighbour face values; affine uses 3 arrays and 4 n^2
  // face values.
  static constexpr int PER = CURVED ? (FE ? 4 * N3 : (4 * N3 > 18 * NT ? 4 * N3 : 18 * NT))
                                    : (FE ? 3 * N3 : (3 * N3 > N3 + 4 * NT ? 3 * N3 : N3 + 4 * NT));
  // per-wavefront copy of the tables indexed by lane: S, Sp, M, l'(0), l'(1)
  static constexpr int LT = 3 * NT + 2 * N;
  static constexpr int LT_S = 0, LT_SP = NT, LT_M = 2 * NT, LT_DL0 = 3 * NT, LT_DL1 = 3 * NT + N;
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
  const T* ltab;  // S, Sp, M, l'(0), l'(1) in device memory (indexed per lane)
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

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of point m on the line of lane t along direction d (x-fastest n^3).
template <int N, int d>
__device__ __forceinline__ int lidx(int t, int m) {
  constexpr int NT = N * N;
  if (d == 0) return m + N * t;
  if (d == 1) return (t % N) + N * m + NT * (t / N);
  return t + NT * m;
}

template <int N, typename T, int d>
__device__ __forceinline__ void read_line(const T* A, int t, T (&x)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) x[m] = A[lidx<N, d>(t, m)];
}
template <int N, typename T, int d>
__device__ __forceinline__ void write_line(T* A, int t, const T (&x)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) A[lidx<N, d>(t, m)] = x[m];
}
// y[q] = sum_m M[q][m] x[m]  (M row-major n x n)
template <int N, typename T>
__device__ __forceinline__ void mat(const T* M, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    T s = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) s += M[q * N + m] * x[m];
    y[q] = s;
  }
}
// y[i] = sum_q M[q][i] x[q]  (transpose)
template <int N, typename T>
__device__ __forceinline__ void matT(const T* M, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) s += M[q * N + i] * x[q];
    y[i] = s;
  }
}

template <int d>
__device__ __forceinline__ int64_t dstride(int Nx, int Ny) {
  return d == 0 ? 1 : (d == 1 ? (int64_t)Nx : (int64_t)Nx * Ny);
}

// Penalty of a face: max of the two element values (Sec. 2), the own value
// on the boundary.
template <int N, typename T>
__device__ __forceinline__ T tau_face(const OpArgs<N, T>& a, int64_t e, bool has, int64_t en) {
  const T te = a.tau[e];
  if (!has) return te;
  const T tn = a.tau[en];
  return te > tn ? te : tn;
}

// Geometry of face (d, s) of the element at ec: the 7 x n^2 block
// (n^T J_L^{-T}, n^T J_R^{-T}, surface weight) of that face, n pointing
// from the lower (L) to the upper (R) element.
template <int N, typename T, int d>
__device__ __forceinline__ const T* face_ptr(const OpArgs<N, T>& a, const int ec[3], int s) {
  constexpr int NT = N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  const int Nd = d == 0 ? a.Nx : (d == 1 ? a.Ny : a.Nz);
  const int Na = da == 0 ? a.Nx : a.Ny;
  const int64_t f = (ec[d] + s) + (int64_t)(Nd + 1) * (ec[da] + (int64_t)Na * ec[db]);
  return a.face[d] + f * 7 * NT;
}

// ------------------------------------------------------------------ curved faces
// Neighbour nodal face data of the two faces of direction d: the end-node
// value P and the normal derivative Q of the neighbour's polynomial on the
// shared face.  F: LDS scratch, 2 values per face.
template <int N, typename T, int d>
__device__ __forceinline__ void nb_nodal(const OpArgs<N, T>& a, T* F, bool act, int t, int64_t e,
                                         const bool has[6]) {
  constexpr int NT = N * N, N3 = N * N * N;
  const int64_t stride = dstride<d>(a.Nx, a.Ny);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    T P = 0, Q = 0;
    if (act && has[f]) {
      const T* un = a.u + (e + (s ? stride : -stride)) * N3;
      T nl[N];
#pragma unroll
      for (int m = 0; m < N; ++m) nl[m] = un[lidx<N, d>(t, m)];
      P = s ? nl[0] : nl[N - 1];
#pragma unroll
      for (int m = 0; m < N; ++m) Q += (s ? a.tab.dl0[m] : a.tab.dl1[m]) * nl[m];
    }
    if (act) {
      F[(2 * f) * NT + t] = P;
      F[(2 * f + 1) * NT + t] = Q;
    }
  }
}

// Second face sweep (along the b direction) of the neighbour data and the
// normal derivative against the own outward normal.  F holds, per face, the
// a-sweep results (value, a-derivative, normal derivative).
template <int N, typename T, int d>
__device__ __forceinline__ void nb_finish(const OpArgs<N, T>& a, const T* F, const T* LT, bool act,
                                          int t, const int ec[3], const bool has[6], T (&un)[6],
                                          T (&dnn)[6]) {
  constexpr int NT = N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  const int ta = t % N, tb = t / N;
  const T* Srow = LT + tb * N;
  const T* Sprow = LT + NT + tb * N;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    un[f] = 0;
    dnn[f] = 0;
    if (!act || !has[f]) continue;
    T u = 0, ga = 0, gb = 0, gd = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const T sv = Srow[q], sp = Sprow[q];
      const int o = ta + N * q;
      const T x1 = F[(3 * f) * NT + o], x2 = F[(3 * f + 1) * NT + o], x3 = F[(3 * f + 2) * NT + o];
      u += sv * x1;
      ga += sv * x2;
      gb += sp * x1;
      gd += sv * x3;
    }
    const T* g = face_ptr<N, T, d>(a, ec, s);
    T cn[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) cn[r] = s ? g[(3 + r) * NT + t] : -g[r * NT + t];
    un[f] = u;
    dnn[f] = cn[d] * gd + cn[da] * ga + cn[db] * gb;
  }
}

// Own traces of the two faces of direction d by extrapolation along the
// d-lines of the Gauss-point data R (u, du/dx, du/dy, du/dz), the flux, and
// the face test coefficients: vt multiplies the test value, gt the test's
// normal derivative (Sec. 2, SIPG flux with the mirror principle).
template <int N, typename T, int d>
__device__ __forceinline__ void own_flux(const OpArgs<N, T>& a, const T* R, bool act, int t, int64_t e,
                                         const int ec[3], const bool has[6], const T (&un)[6],
                                         const T (&dnn)[6], T (&vt)[6], T (&gt)[6]) {
  constexpr int N3 = N * N * N, NT = N * N;
  const auto& tab = a.tab;
  const int64_t stride = dstride<d>(a.Nx, a.Ny);
  T uq[N], g0[N], g1[N], g2[N];
  if (act) {
    read_line<N, T, d>(R, t, uq);
    read_line<N, T, d>(R + N3, t, g0);
    read_line<N, T, d>(R + 2 * N3, t, g1);
    read_line<N, T, d>(R + 3 * N3, t, g2);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    vt[f] = 0;
    gt[f] = 0;
    if (!act) continue;
    if (!has[f] && ((a.bcmask >> f) & 1)) continue;  // Neumann: no face term
    T uo = 0, h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T l = s ? tab.lg1[m] : tab.lg0[m];
      uo += l * uq[m];
      h0 += l * g0[m];
      h1 += l * g1[m];
      h2 += l * g2[m];
    }
    const T* g = face_ptr<N, T, d>(a, ec, s);
    T co[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) co[r] = s ? g[r * NT + t] : -g[(3 + r) * NT + t];
    const T dA = g[6 * NT + t];
    const T dno = co[0] * h0 + co[1] * h1 + co[2] * h2;
    const T tauF = tau_face(a, e, has[f], e + (s ? stride : -stride));
    T jump, avg;
    if (has[f]) {
      jump = uo - un[f];
      avg = T(0.5) * (dno + dnn[f]);
    } else {  // Dirichlet mirror: u+ = -u-, grad u+ = grad u-
      jump = T(2) * uo;
      avg = dno;
    }
    vt[f] = (tauF * jump - avg) * dA;
    gt[f] = T(-0.5) * jump * dA;
  }
}

// Add the face tests of direction d to the d-lines of the integration
// arrays (vq: test value, fx/fy/fz: test reference gradient).
template <int N, typename T, int d>
__device__ __forceinline__ void inject(const OpArgs<N, T>& a, const int ec[3], int t, const T (&vt)[6],
                                       const T (&gt)[6], T (&vq)[N], T (&fx)[N], T (&fy)[N], T (&fz)[N]) {
  constexpr int NT = N * N;
  const auto& tab = a.tab;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    const T* g = face_ptr<N, T, d>(a, ec, s);
    T c[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) c[r] = (s ? g[r * NT + t] : -g[(3 + r) * NT + t]) * gt[f];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T l = s ? tab.lg1[m] : tab.lg0[m];
      vq[m] += l * vt[f];
      fx[m] += l * c[0];
      fy[m] += l * c[1];
      fz[m] += l * c[2];
    }
  }
}

// ------------------------------------------------------------------ affine faces
// Nodal face terms of direction d added to the x-line accumulator vacc.
// With n^T J^{-T} = +-e_d / h_d on both sides and surface weight
// h_a h_b w_a w_b, the flux reduces to the plane term tau [u] - c {du/dn}
// and the normal-derivative term -c/2 [u], each taken through the face mass
// matrix M (x) M.  A: own nodal u; F: LDS scratch of 4 n^2.
template <int N, typename T, int d>
__device__ __forceinline__ void affine_faces(const OpArgs<N, T>& a, const T* A, T* F, const T* LT,
                                             bool act, int t, int64_t e, const bool has[6],
                                             T (&vacc)[N]) {
  constexpr int NT = N * N, N3 = N * N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  const auto& tab = a.tab;
  const int ta = t % N, tbb = t / N;
  const int64_t stride = dstride<d>(a.Nx, a.Ny);
  if (act) {
    T line[N];
    read_line<N, T, d>(A, t, line);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * d + s;
      const bool neu = !has[f] && ((a.bcmask >> f) & 1);
      const T Po = line[s * (N - 1)];
      T Qo = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) Qo += (s ? tab.dl1[m] : tab.dl0[m]) * line[m];
      T Pj, Qs;
      if (has[f]) {
        const T* un = a.u + (e + (s ? stride : -stride)) * N3;
        T nl[N];
#pragma unroll
        for (int m = 0; m < N; ++m) nl[m] = un[lidx<N, d>(t, m)];
        T Qn = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) Qn += (s ? tab.dl0[m] : tab.dl1[m]) * nl[m];
        Pj = Po - (s ? nl[0] : nl[N - 1]);
        Qs = Qo + Qn;
      } else {
        Pj = neu ? T(0) : T(2) * Po;
        Qs = neu ? T(0) : T(2) * Qo;
      }
      const T cd = (s ? T(1) : T(-1)) / a.h[d];
      const T tauF = tau_face(a, e, has[f], e + (s ? stride : -stride));
      F[(2 * s) * NT + t] = tauF * Pj - T(0.5) * cd * Qs;
      F[(2 * s + 1) * NT + t] = T(-0.5) * cd * Pj;
    }
  }
  wave_sync();
  T Z[4] = {0, 0, 0, 0};
  if (act)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < N; ++q) Z[c] += LT[2 * NT + ta * N + q] * F[c * NT + q + N * tbb];
  wave_sync();
  if (act)
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c * NT + t] = Z[c];
  wave_sync();
  T W[4] = {0, 0, 0, 0};
  if (act) {
    const T hab = a.h[da] * a.h[db];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int q = 0; q < N; ++q) W[c] += LT[2 * NT + tbb * N + q] * F[c * NT + ta + N * q];
      W[c] *= hab;
    }
  }
  wave_sync();
  if (act)
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c * NT + t] = W[c];
  wave_sync();
  // F[(2s) n^2 + node]: plane term at the end node; F[(2s+1) n^2 + node]:
  // weight of l_i'(s) along the normal line.  Add into this lane's x-line.
  if (act) {
    const int j = t % N, l = t / N;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* Pv = F + (2 * s) * NT;
      const T* Qv = F + (2 * s + 1) * NT;
      const int endp = s * (N - 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (d == 0) {
          vacc[i] += (i == endp ? Pv[t] : T(0)) + (s ? tab.dl1[i] : tab.dl0[i]) * Qv[t];
        } else if (d == 1) {
          vacc[i] += (j == endp ? Pv[i + N * l] : T(0)) + LT[3 * NT + s * N + j] * Qv[i + N * l];
        } else {
          vacc[i] += (l == endp ? Pv[i + N * j] : T(0)) + LT[3 * NT + s * N + l] * Qv[i + N * j];
        }
      }
    }
  }
  wave_sync();
}

// ------------------------------------------------------------------ operator
template <int N, typename T, bool CURVED, bool FE, int MODE>
__global__ void __launch_bounds__(256) op_kernel(const OpArgs<N, T> a) {
  using C = Cfg<N, CURVED, FE>;
  constexpr int NT = C::NT, N3 = C::N3, EW = C::EW, PER = C::PER;
  __shared__ T smem[C::WAVES * (EW * PER + C::LT)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int le = lane / NT, t = lane - le * NT;
  const int64_t e0 = (int64_t)xcd_block() * C::EB + (int64_t)wave * EW;  // first element of the wave
  const int64_t e = e0 + le;
  const bool act = (le < EW) && (e < a.nel);
  T* const W0 = smem + wave * (EW * PER + C::LT);  // this wavefront's LDS
  T* const R = W0 + (le < EW ? le : 0) * PER;
  T* const LT = W0 + EW * PER;
  const auto& tab = a.tab;
  for (int i = lane; i < C::LT; i += 64) LT[i] = a.ltab[i];
  int ec[3] = {0, 0, 0};
  bool has[6] = {false, false, false, false, false, false};
  if (act) {
    ec[0] = (int)(e % a.Nx);
    const int64_t r = e / a.Nx;
    ec[1] = (int)(r % a.Ny);
    ec[2] = (int)(r / a.Ny);
    has[0] = ec[0] > 0;
    has[1] = ec[0] + 1 < a.Nx;
    has[2] = ec[1] > 0;
    has[3] = ec[1] + 1 < a.Ny;
    has[4] = ec[2] > 0;
    has[5] = ec[2] + 1 < a.Nz;
  }
  const int64_t left = a.nel - e0;
  const int nload = (int)(left <= 0 ? 0 : (left < EW ? left : EW)) * N3;
  const int ta = t % N, tbb = t / N;

  // ---- neighbour traces (curved DG), before the own data occupies LDS
  T un[6], dnn[6];
  if constexpr (CURVED && !FE) {
    nb_nodal<N, T, 0>(a, R, act, t, e, has);
    nb_nodal<N, T, 1>(a, R, act, t, e, has);
    nb_nodal<N, T, 2>(a, R, act, t, e, has);
    wave_sync();
    T X[18];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      X[3 * f] = X[3 * f + 1] = X[3 * f + 2] = 0;
      if (act)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = LT[ta * N + q], sp = LT[NT + ta * N + q];
          const T p = R[(2 * f) * NT + q + N * tbb], qq = R[(2 * f + 1) * NT + q + N * tbb];
          X[3 * f] += sv * p;
          X[3 * f + 1] += sp * p;
          X[3 * f + 2] += sv * qq;
        }
    }
    wave_sync();
    if (act)
#pragma unroll
      for (int c = 0; c < 18; ++c) R[c * NT + t] = X[c];
    wave_sync();
    nb_finish<N, T, 0>(a, R, LT, act, t, ec, has, un, dnn);
    nb_finish<N, T, 1>(a, R, LT, act, t, ec, has, un, dnn);
    nb_finish<N, T, 2>(a, R, LT, act, t, ec, has, un, dnn);
    wave_sync();
  }

  // ---- own element data into LDS (coalesced per wavefront)
  if constexpr (!FE) {
    const T* src = a.u + e0 * N3;
    for (int idx = lane; idx < nload; idx += 64) {
      const int li = idx / N3;
      W0[li * PER + (idx - li * N3)] = src[idx];
    }
  } else {
    constexpr int k = N - 1;
    const int64_t Mx = (int64_t)a.Nx * k + 1, My = (int64_t)a.Ny * k + 1, Mz = (int64_t)a.Nz * k + 1;
    for (int idx = lane; idx < nload; idx += 64) {
      const int li = idx / N3, p = idx - li * N3;
      const int64_t ee = e0 + li;
      const int64_t gx = (ee % a.Nx) * k + p % N;
      const int64_t rr = ee / a.Nx;
      const int64_t gy = (rr % a.Ny) * k + (p / N) % N;
      const int64_t gz = (rr / a.Ny) * k + p / NT;
      const int m = a.bcmask;
      const bool fixed = (gx == 0 && !(m & 1)) || (gx == Mx - 1 && !(m & 2)) || (gy == 0 && !(m & 4)) ||
                         (gy == My - 1 && !(m & 8)) || (gz == 0 && !(m & 16)) || (gz == Mz - 1 && !(m & 32));
      W0[li * PER + p] = fixed ? T(0) : a.u[gx + Mx * (gy + My * gz)];
    }
  }
  wave_sync();

  T* const A = R;
  T* const B = R + N3;
  T* const Cc = R + 2 * N3;
  T v[N];

  if constexpr (!CURVED) {
    // ---- affine: faces in nodal space, cell as sum_d c_d K_d (x) M (x) M
    T vacc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) vacc[i] = 0;
    if constexpr (!FE) {
      affine_faces<N, T, 0>(a, A, B, LT, act, t, e, has, vacc);
      affine_faces<N, T, 1>(a, A, B, LT, act, t, e, has, vacc);
      affine_faces<N, T, 2>(a, A, B, LT, act, t, e, has, vacc);
    }
    const T cx = a.h[1] * a.h[2] / a.h[0], cy = a.h[0] * a.h[2] / a.h[1], cz = a.h[0] * a.h[1] / a.h[2];
    if (act) {  // z: p = M u, q = K u
      T x[N], p[N], q[N];
      read_line<N, T, 2>(A, t, x);
      mat<N, T>(tab.M, x, p);
      mat<N, T>(tab.K, x, q);
      write_line<N, T, 2>(B, t, p);
      write_line<N, T, 2>(Cc, t, q);
    }
    wave_sync();
    if (act) {  // y: r = M p, s = cy K p + cz M q
      T p[N], q[N], r[N], s1[N], s2[N];
      read_line<N, T, 1>(B, t, p);
      read_line<N, T, 1>(Cc, t, q);
      mat<N, T>(tab.M, p, r);
      mat<N, T>(tab.K, p, s1);
      mat<N, T>(tab.M, q, s2);
#pragma unroll
      for (int m = 0; m < N; ++m) s1[m] = cy * s1[m] + cz * s2[m];
      write_line<N, T, 1>(B, t, r);
      write_line<N, T, 1>(Cc, t, s1);
    }
    wave_sync();
    if (act) {  // x: v = cx K r + M s
      T r[N], s[N], v1[N], v2[N];
      read_line<N, T, 0>(B, t, r);
      read_line<N, T, 0>(Cc, t, s);
      mat<N, T>(tab.K, r, v1);
      mat<N, T>(tab.M, s, v2);
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = cx * v1[m] + v2[m] + vacc[m];
    }
  } else {
    T* const Dg = R + 3 * N3;
    // ---- curved: interpolation to Gauss points, x then y then z
    if (act) {
      T x[N], y[N];
      read_line<N, T, 0>(A, t, x);
      mat<N, T>(tab.S, x, y);
      write_line<N, T, 0>(A, t, y);
    }
    wave_sync();
    if (act) {
      T x[N], y[N];
      read_line<N, T, 1>(A, t, x);
      mat<N, T>(tab.S, x, y);
      write_line<N, T, 1>(A, t, y);
    }
    wave_sync();
    if (act) {
      T x[N], uq[N], gz[N];
      read_line<N, T, 2>(A, t, x);
      mat<N, T>(tab.S, x, uq);
      mat<N, T>(tab.D, uq, gz);
      write_line<N, T, 2>(A, t, uq);
      write_line<N, T, 2>(Dg, t, gz);
    }
    wave_sync();
    if (act) {  // collocation derivatives in x (-> B) and y (-> Cc)
      T x[N], y[N];
      read_line<N, T, 0>(A, t, x);
      mat<N, T>(tab.D, x, y);
      write_line<N, T, 0>(B, t, y);
      read_line<N, T, 1>(A, t, x);
      mat<N, T>(tab.D, x, y);
      write_line<N, T, 1>(Cc, t, y);
    }
    wave_sync();
    // ---- face fluxes (DG): own traces by extrapolation
    T vt[6], gt[6];
    if constexpr (!FE) {
      own_flux<N, T, 0>(a, R, act, t, e, ec, has, un, dnn, vt, gt);
      own_flux<N, T, 1>(a, R, act, t, e, ec, has, un, dnn, vt, gt);
      own_flux<N, T, 2>(a, R, act, t, e, ec, has, un, dnn, vt, gt);
      wave_sync();
    }
    // ---- quadrature-point operator on z-lines, z-face tests
    if (act) {
      T vq[N], fx[N], fy[N], fz[N];
      const T* G = a.metric + e * 6 * N3 + t;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int o = t + NT * m;
        const T gx = B[o], gy = Cc[o], g3 = Dg[o];
        const T* Gm = G + NT * m;
        const T g00 = Gm[0], g11 = Gm[N3], g22 = Gm[2 * N3], g01 = Gm[3 * N3], g02 = Gm[4 * N3],
                g12 = Gm[5 * N3];
        fx[m] = g00 * gx + g01 * gy + g02 * g3;
        fy[m] = g01 * gx + g11 * gy + g12 * g3;
        fz[m] = g02 * gx + g12 * gy + g22 * g3;
        vq[m] = 0;
      }
      if constexpr (!FE) inject<N, T, 2>(a, ec, t, vt, gt, vq, fx, fy, fz);
      if constexpr (!FE) write_line<N, T, 2>(A, t, vq);
      write_line<N, T, 2>(B, t, fx);
      write_line<N, T, 2>(Cc, t, fy);
      write_line<N, T, 2>(Dg, t, fz);
    }
    wave_sync();
    if constexpr (!FE) {  // x-face tests along x-lines
      if (act) {
        T vq[N], fx[N], fy[N], fz[N];
        read_line<N, T, 0>(A, t, vq);
        read_line<N, T, 0>(B, t, fx);
        read_line<N, T, 0>(Cc, t, fy);
        read_line<N, T, 0>(Dg, t, fz);
        inject<N, T, 0>(a, ec, t, vt, gt, vq, fx, fy, fz);
        write_line<N, T, 0>(A, t, vq);
        write_line<N, T, 0>(B, t, fx);
        write_line<N, T, 0>(Cc, t, fy);
        write_line<N, T, 0>(Dg, t, fz);
      }
      wave_sync();
    }
    if (act) {  // y-face tests, then integration in y
      T fx[N], fy[N], fz[N], ay[N], by[N], cy[N], w2[N];
      read_line<N, T, 1>(B, t, fx);
      read_line<N, T, 1>(Cc, t, fy);
      read_line<N, T, 1>(Dg, t, fz);
      if constexpr (!FE) {
        T vq[N];
        read_line<N, T, 1>(A, t, vq);
        inject<N, T, 1>(a, ec, t, vt, gt, vq, fx, fy, fz);
        matT<N, T>(tab.S, vq, cy);
      }
      matT<N, T>(tab.S, fx, ay);
      matT<N, T>(tab.S, fz, by);
      matT<N, T>(tab.Sp, fy, w2);
#pragma unroll
      for (int m = 0; m < N; ++m) cy[m] = FE ? w2[m] : cy[m] + w2[m];
      write_line<N, T, 1>(A, t, ay);
      write_line<N, T, 1>(B, t, by);
      write_line<N, T, 1>(Cc, t, cy);
    }
    wave_sync();
    if (act) {  // integration in z
      T ay[N], by[N], cy[N], az[N], bz[N], w2[N];
      read_line<N, T, 2>(A, t, ay);
      read_line<N, T, 2>(B, t, by);
      read_line<N, T, 2>(Cc, t, cy);
      matT<N, T>(tab.S, ay, az);
      matT<N, T>(tab.Sp, by, bz);
      matT<N, T>(tab.S, cy, w2);
#pragma unroll
      for (int m = 0; m < N; ++m) bz[m] += w2[m];
      write_line<N, T, 2>(A, t, az);
      write_line<N, T, 2>(B, t, bz);
    }
    wave_sync();
    if (act) {  // integration in x
      T az[N], bz[N], w2[N];
      read_line<N, T, 0>(A, t, az);
      read_line<N, T, 0>(B, t, bz);
      matT<N, T>(tab.Sp, az, v);
      matT<N, T>(tab.S, bz, w2);
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] += w2[m];
    }
  }
  wave_sync();
  if (act) write_line<N, T, 0>(A, t, v);
  wave_sync();

  // ---- coalesced epilogue over the wavefront's elements
  const int64_t gbase = e0 * N3;
  double acc = 0.0;
  for (int idx = lane; idx < nload; idx += 64) {
    const int li = idx / N3;
    const T val = W0[li * PER + (idx - li * N3)];
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
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) a.partials[(int64_t)blockIdx.x * C::WAVES + wave] = acc;
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
  a.ltab = (const T*)L->ltab();
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
  using C = Cfg<N, CURVED, FE>;
  OpArgs<N, T> a = make_args<N, T>(L);
  a.u = (const T*)u;
  a.out = (T*)(FE ? L->scratch() : out);
  a.b = (const T*)b;
  a.xold = (const T*)xold;
  a.sigma = (T)sigma;
  a.theta = (T)theta;
  const int64_t nb = (L->n_el + C::EB - 1) / C::EB;
  if (nb > INT32_MAX / C::WAVES) return fail(HMG_ERR_UNSUPPORTED, "mesh too large for one launch");
  // one partial per wavefront; the level's partials buffer holds n_el + 64
  if (nparts) *nparts = (int)nb * C::WAVES;
  dim3 grid((unsigned)nb), block(64 * C::WAVES);
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
