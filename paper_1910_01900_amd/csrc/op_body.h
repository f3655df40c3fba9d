// Device side of the matrix-free SIPG / continuous-FE Laplace operator for
// gfx950 (Sec. 4, eq:MatrixFreeAbstractNotation): workgroup geometry,
// helpers and the per-group operator body shared by the single-mesh and
// the multi-mesh kernels.
//
// Work decomposition: lanes form groups (a wavefront, or at n = 6 the
// whole 256-lane workgroup); a group owns EW = lanes / n^2 elements outright
// (n^2 lanes per element) and a private LDS region, and all exchanges
// between lanes stay inside the group.  Wavefront groups separate their
// phases by wavefront fences instead of workgroup barriers, so the four
// wavefronts of a workgroup progress independently (the latency of one
// hides behind the others).  At n = 6 a wavefront would hold one element
// on 36 of its 64 lanes; the workgroup group holds 7 on 252 of 256 lanes,
// with workgroup barriers between phases (FP64 apply 13% faster, FP32 11%;
// at n = 5 and 7, 78% and 77% of the lanes work either way and the
// workgroup group measured no faster).  Lane t of an element owns one line
// of n points along the direction of the current phase (x-lines:
// t = j + n*l, y-lines: t = i + n*l, z-lines: t = i + n*j), so every 1-D
// contraction is a register-only loop; LDS only changes the direction.
//
// 1-D contractions use the even-odd decomposition of the centro-symmetric
// (S, M, K) and skew (D, Sp) tables (Sec. 4 sum factorization), with the
// packed coefficients in scalar registers, loaded per phase from a
// device-memory table so that only one phase's coefficients are live.
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
#pragma once

#include "hmg_internal.h"

namespace hmg {

template <int N, bool CURVED, bool FE>
struct Cfg {
  static constexpr int NT = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int AS = lds_array_size(N);  // LDS values of one n^3 array (padded)
  static constexpr int WAVES = kOpWaves;
  static constexpr int GL = op_group_lanes(N);        // lanes of a group (64 or the workgroup)
  static constexpr int GROUPS = 64 * WAVES / GL;      // groups per workgroup
  static constexpr int EW = op_elems_per_group(N);    // elements per group
  static constexpr int EB = op_elems_per_block(N);    // elements per workgroup
  static_assert(EB == EW * GROUPS, "workgroup geometry");
  // LDS values per element: curved DG uses 4 arrays (value/flux x, y, z)
  // and 18 n^2 neighbour face values, curved FE 3 (its z-derivative stays in
  // registers); affine uses 3 arrays and 4 n^2 face values.
  // Padded to PER = 9 (mod 16) values so that the lines of the elements
  // sharing a wavefront fall on different LDS banks.
  static constexpr int PER0 = CURVED ? (FE ? 3 * AS : (4 * AS > 18 * NT ? 4 * AS : 18 * NT))
                                     : (FE ? 3 * AS : (3 * AS > AS + 4 * NT ? 3 * AS : AS + 4 * NT));
  static constexpr int PER = PER0 + ((9 - PER0 % 16) + 16) % 16;
  static constexpr int LT = TabOff(N).lane_size();
  // minimum waves per SIMD the register allocation must allow (n >= 7: LDS
  // already limits residency to two)
  static constexpr int WPE = N >= 7 ? 2 : 3;  // per-wavefront copy of S, Sp, M, l'(0), l'(1)
};

// Minimum waves per SIMD the register allocation of the (N, T) kernel must
// allow: Cfg::WPE, and four for the FP32 curvilinear DG kernels at n >= 7,
// whose LDS use allows four workgroups per CU.
template <int N, typename T, bool CURVED, bool FE>
constexpr int op_wpe() {
  return (CURVED && !FE && N >= 7 && sizeof(T) == 4) ? 4 : Cfg<N, CURVED, FE>::WPE;
}

// Whether the epilogue of MODE reads the input vector again (Chebyshev
// update, u.(A u)) and the group keeps its own input values in LDS
// instead of reading them from memory a second time: only where the extra
// LDS does not lower residency (workgroups per CU from 160 KB of LDS,
// against the register limit: WPE for the FP64 curvilinear kernels, about
// five otherwise).
template <int N, typename T, bool CURVED, bool FE, int MODE>
constexpr bool keeps_input() {
  if (FE || (MODE != OP_CHEB && MODE != OP_DOT)) return false;
  using C = Cfg<N, CURVED, FE>;
  constexpr int base = C::GROUPS * (C::EW * C::PER + C::LT) * (int)sizeof(T);
  constexpr int extra = C::GROUPS * C::EW * C::N3 * (int)sizeof(T);
  constexpr int vgpr_blocks = (CURVED && sizeof(T) == 8) ? C::WPE : 5;
  constexpr int b0 = 163840 / base, b1 = 163840 / (base + extra);
  return (b1 < vgpr_blocks ? b1 : vgpr_blocks) == (b0 < vgpr_blocks ? b0 : vgpr_blocks);
}
// LDS values of one group: EW elements of PER, the lane tables, and the
// kept input values.
template <int N, typename T, bool CURVED, bool FE, int MODE>
constexpr int op_group_lds() {
  using C = Cfg<N, CURVED, FE>;
  return C::EW * C::PER + C::LT + (keeps_input<N, T, CURVED, FE, MODE>() ? C::EW * C::N3 : 0);
}

// ------------------------------------------------------------------ helpers
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// A copy of p the compiler cannot trace back: loads through it are issued
// where it is made (scalar loads, uniform address), so table coefficients
// live in scalar registers for one phase only.
template <typename T>
__device__ __forceinline__ cptr<T> fresh(const T* p) {
  cptr<T> c = (cptr<T>)(uintptr_t)p;
  asm volatile("" : "+s"(c)::"memory");
  return c;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical workgroups so that neighbouring elements are
// processed on the same XCD (one L2).
__device__ __forceinline__ int xcd_block() {
  int nb = gridDim.x, x = blockIdx.x & 7, y = blockIdx.x >> 3;
  int per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + y;
}

// Work items of logical workgroup b: up to EB consecutive items from the
// returned first one; *count is how many (fewer at the end of the launch,
// and at the end of an x-row).  With a.rowchunks = ceil(Nx / EB) chunks per
// x-row (one vector), rows are visited in y-tiles of tile_y rows, z before
// y inside a tile: the x, y and z neighbours of an element are then
// processed close in time (a few dozen workgroups apart) and the shared
// face geometry and neighbour values are still in L2.  A row's last chunk
// holds the Nx mod EB elements left over (if any).
template <typename T>
__device__ __forceinline__ int64_t block_chunk(const OpArgs<T>& a, int b, int eb, int* count) {
  const int R = a.rowchunks;
  if (R == 0) {
    const int64_t first = (int64_t)b * eb, left = a.nel * a.nrhs - first;
    *count = left < eb ? (int)left : eb;
    return first;
  }
  // 32-bit: chunk counts are below 2^31 (checked at launch)
  const unsigned TY = a.tile_y, full = (unsigned)R * a.Nz * TY;
  const unsigned ty = (unsigned)b / full;
  const unsigned th = min(TY, a.Ny - ty * TY);
  const unsigned bp = (unsigned)b - ty * full;
  const unsigned r = bp / R, cx = bp - r * R;
  const unsigned z = r / th, yi = r - z * th;
  const int x0 = (int)cx * eb;
  *count = a.Nx - x0 < eb ? a.Nx - x0 : eb;
  return x0 + (int64_t)a.Nx * ((ty * TY + yi) + (int64_t)a.Ny * z);
}

// Pin a value in registers at this point: computations that feed stores
// after a wave_sync() are otherwise sunk past it, which keeps all of their
// LDS inputs live across the fence.
template <typename T>
__device__ __forceinline__ void pin(T& x) {
  asm volatile("" : "+v"(x));
}

// Order LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// Order LDS traffic between the lanes of a group of GL lanes (a wavefront,
// or the whole workgroup).
template <int GL>
__device__ __forceinline__ void group_sync() {
  if constexpr (GL == 64) {
    wave_sync();
  } else {
    __syncthreads();
  }
}

// Index of point m on the line of lane t along direction d (x-fastest n^3).
template <int N, int d>
__device__ __forceinline__ int lidx(int t, int m) {
  constexpr int NT = N * N;
  if (d == 0) return m + N * t;
  if (d == 1) return (t % N) + N * m + NT * (t / N);
  return t + NT * m;
}

// Position of node (i, j, l) of an element in its LDS arrays.  For n = 8
// the plain order puts the lanes of an x-line access (one i, all j, l) on
// 8 banks and those of a y-line access on 8 or 16; rows padded to 9 values
// and planes to 72 put x- and y-line accesses on distinct banks and z-line
// accesses at most two to a bank (4- and 8-byte values, 32 or 64 banks,
// checked exhaustively on the host), and every point of a line is its
// lane's base address plus a constant, an instruction offset.  Other
// degrees keep the plain x-fastest order, whose line accesses are at most
// two-way conflicted.
template <int N>
__device__ __forceinline__ int vpos(int i, int j, int l) {
  if constexpr (N == 8)
    return i + 9 * j + 72 * l;
  else
    return i + N * j + N * N * l;
}
// LDS position of node p (x-fastest index) of an element.
template <int N>
__device__ __forceinline__ int vpos_of(int p) {
  if constexpr (N == 8)
    return vpos<N>(p & 7, (p >> 3) & 7, p >> 6);
  else
    return p;
}
// LDS position of point m on the line of lane t along direction d.
template <int N, int d>
__device__ __forceinline__ int sidx(int t, int m) {
  if constexpr (N != 8) return lidx<N, d>(t, m);
  if constexpr (d == 0) return vpos<N>(m, t % N, t / N);
  if constexpr (d == 1) return vpos<N>(t % N, m, t / N);
  return vpos<N>(t % N, t / N, m);
}

template <int N, typename T, int d>
__device__ __forceinline__ void read_line(const T* A, int t, T (&x)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) x[m] = A[sidx<N, d>(t, m)];
}
template <int N, typename T, int d>
__device__ __forceinline__ void write_line(T* A, int t, const T (&x)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) A[sidx<N, d>(t, m)] = x[m];
}

// y = A x with A given by its even-odd packing c (see TabOff); SIG = +1 for
// centro-symmetric, -1 for skew tables.
template <int N, typename T, int SIG>
__device__ __forceinline__ void eo_apply(cptr<T> c, const T (&x)[N], T (&y)[N]) {
  constexpr int h = N / 2;
  constexpr bool odd = N & 1;
  T xe[h > 0 ? h : 1], xo[h > 0 ? h : 1];
#pragma unroll
  for (int i = 0; i < h; ++i) {
    xe[i] = x[i] + x[N - 1 - i];
    xo[i] = x[i] - x[N - 1 - i];
  }
#pragma unroll
  for (int q = 0; q < h; ++q) {
    T ye = c[q * h] * xe[0];
    T yo = c[h * h + q * h] * xo[0];
#pragma unroll
    for (int i = 1; i < h; ++i) {
      ye += c[q * h + i] * xe[i];
      yo += c[h * h + q * h + i] * xo[i];
    }
    if (odd) ye += c[2 * h * h + q] * x[h];
    y[q] = ye + yo;
    y[N - 1 - q] = SIG > 0 ? ye - yo : yo - ye;
  }
  if (odd) {
    T ym = SIG > 0 ? c[2 * h * h + 2 * h] * x[h] : T(0);
#pragma unroll
    for (int i = 0; i < h; ++i) ym += c[2 * h * h + h + i] * (SIG > 0 ? xe[i] : xo[i]);
    y[h] = ym;
  }
}

template <int d>
__device__ __forceinline__ int64_t dstride(int Nx, int Ny) {
  return d == 0 ? 1 : (d == 1 ? (int64_t)Nx : (int64_t)Nx * Ny);
}

// Penalty of a face: max of the two element values (Sec. 2), the own value
// on the boundary.
template <typename T>
__device__ __forceinline__ T tau_face(T te, T tn, bool has) {
  return has ? (te > tn ? te : tn) : te;
}

// Per element: a valid element index (lanes without an element use a
// clamped one, so that every address stays inside the arrays and loads need
// no branch), neighbour flags (bit f for face f = 2d + s) and, per direction,
// the index of the lower face in that direction's face array.
struct ElemInfo {
  int64_t e;
  int hb;
  int fidx[3];
};

// x / d for x < 2^31 from the host's FP64 inv = 1/d: (x + 1/2) / d lies at
// least 1/(2d) from an integer and the two rounded FP64 operations move it by
// less than 2^-20 / d, so truncation gives the exact quotient (three VALU
// instructions instead of an integer division by a run-time value).
__device__ __forceinline__ unsigned exact_div(unsigned x, double inv) {
  return (unsigned)(((double)x + 0.5) * inv);
}

template <typename T>
__device__ __forceinline__ ElemInfo elem_info(const OpArgs<T>& a, int64_t e) {
  ElemInfo I;
  I.e = e < a.nel ? e : a.nel - 1;
  // element counts are below 2^31 (checked at level creation)
  const unsigned ue = (unsigned)I.e, r = exact_div(ue, a.inv_nx), uz = exact_div(r, a.inv_ny);
  const int ex = (int)(ue - r * a.Nx), ey = (int)(r - uz * a.Ny), ez = (int)uz;
  I.hb = (ex > 0) | ((ex + 1 < a.Nx) << 1) | ((ey > 0) << 2) | ((ey + 1 < a.Ny) << 3) | ((ez > 0) << 4) |
         ((ez + 1 < a.Nz) << 5);
  // faces of direction d are numbered (pos_d) + (N_d + 1) (pos_a + N_a pos_b)
  I.fidx[0] = ex + (a.Nx + 1) * (ey + a.Ny * ez);
  I.fidx[1] = ey + (a.Ny + 1) * (ex + a.Nx * ez);
  I.fidx[2] = ez + (a.Nz + 1) * (ex + a.Nx * ey);
  return I;
}

__device__ __forceinline__ bool has_nb(const ElemInfo& I, int f) { return (I.hb >> f) & 1; }

// Neighbour across face (d, s), or the element itself on the boundary (its
// data is then loaded but not used).
template <int d, typename T>
__device__ __forceinline__ int64_t nb_elem(const OpArgs<T>& a, const ElemInfo& I, int s) {
  return has_nb(I, 2 * d + s) ? I.e + (s ? dstride<d>(a.Nx, a.Ny) : -dstride<d>(a.Nx, a.Ny)) : I.e;
}

// Geometry block of face (d, s) at face point t: 7 x n^2 values
// (n^T J_L^{-T}, n^T J_R^{-T}, surface weight), n pointing from the lower (L)
// to the upper (R) element.
template <int N, typename T, int d>
__device__ __forceinline__ const T* face_ptr(const OpArgs<T>& a, const ElemInfo& I, int s, int t) {
  return a.face[d] + (int64_t)(I.fidx[d] + s) * (7 * N * N) + t;
}

// n^T J^{-T} of face (d, s) at face point t with n the own outward normal,
// of the own side (OWN) or of the neighbour side.
template <int N, typename T, int d, bool OWN>
__device__ __forceinline__ void face_metric(const OpArgs<T>& a, const ElemInfo& I, int s, int t, T (&c)[3]) {
  constexpr int NT = N * N;
  const T* g = face_ptr<N, T, d>(a, I, s, t);
  const int off = (OWN == (s == 1)) ? 0 : 3;
#pragma unroll
  for (int r = 0; r < 3; ++r) c[r] = s ? g[(off + r) * NT] : -g[(off + r) * NT];
}

// Neighbour-side n^T J^{-T} of all six faces at face point t.
template <int N, typename T>
__device__ __forceinline__ void nb_face_metric(const OpArgs<T>& a, const ElemInfo& I, int t, T (&cn)[6][3]) {
  face_metric<N, T, 0, false>(a, I, 0, t, cn[0]);
  face_metric<N, T, 0, false>(a, I, 1, t, cn[1]);
  face_metric<N, T, 1, false>(a, I, 0, t, cn[2]);
  face_metric<N, T, 1, false>(a, I, 1, t, cn[3]);
  face_metric<N, T, 2, false>(a, I, 0, t, cn[4]);
  face_metric<N, T, 2, false>(a, I, 1, t, cn[5]);
}

// ------------------------------------------------------------------ curved faces
// Neighbour lines of the two faces of direction d (global memory).
template <int N, typename T, int d>
__device__ __forceinline__ void load_nb_lines(const OpArgs<T>& a, const T* ub, const ElemInfo& I, int t,
                                              T (&l0)[N], T (&l1)[N]) {
  constexpr int N3 = N * N * N;
  const T* u0 = ub + nb_elem<d>(a, I, 0) * N3;
  const T* u1 = ub + nb_elem<d>(a, I, 1) * N3;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    l0[m] = u0[lidx<N, d>(t, m)];
    l1[m] = u1[lidx<N, d>(t, m)];
  }
}

// Second face sweep (along the b direction) of the neighbour data and the
// normal derivative against the own outward normal.  F holds, per face, the
// a-sweep results (value, a-derivative, normal derivative); cn is the
// neighbour-side metric of the faces.
template <int N, typename T, int d>
__device__ __forceinline__ void nb_finish(const T* F, const T* LT, int t, const ElemInfo& I,
                                          const T (&cn)[6][3], T (&un)[6], T (&dnn)[6]) {
  constexpr int NT = N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  const int ta = t % N, tb = t / N;
  const T* Srow = LT + tb * N;
  const T* Sprow = LT + NT + tb * N;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
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
    const bool hf = has_nb(I, f);
    un[f] = hf ? u : T(0);
    dnn[f] = hf ? cn[f][d] * gd + cn[f][da] * ga + cn[f][db] * gb : T(0);
  }
}

// Global data of the two faces of direction d at face point t: own-side
// n^T J^{-T} (co), surface weights (dA) and the neighbours' penalties (tn).
template <typename T>
struct OwnFace {
  T co[2][3], dA[2], tn[2];
};

template <int N, typename T, int d>
__device__ __forceinline__ OwnFace<T> load_own_face(const OpArgs<T>& a, const ElemInfo& I, int t) {
  constexpr int NT = N * N;
  OwnFace<T> F;
  face_metric<N, T, d, true>(a, I, 0, t, F.co[0]);
  face_metric<N, T, d, true>(a, I, 1, t, F.co[1]);
  F.dA[0] = face_ptr<N, T, d>(a, I, 0, t)[6 * NT];
  F.dA[1] = face_ptr<N, T, d>(a, I, 1, t)[6 * NT];
  F.tn[0] = a.tau[nb_elem<d>(a, I, 0)];
  F.tn[1] = a.tau[nb_elem<d>(a, I, 1)];
  return F;
}

// Own traces of the two faces of direction d by extrapolation along the
// d-lines of the Gauss-point data R (u, du/dx, du/dy, du/dz), the flux, and
// the face test coefficients: vt multiplies the test value, gt the test's
// normal derivative (Sec. 2, SIPG flux with the mirror principle).  F holds
// the faces' global data (loaded a phase earlier), te the element's penalty.
// PRE: also the products gc of the own-side metric with gt.
template <int N, typename T, int d, bool PRE>
__device__ __forceinline__ void own_flux(const OpArgs<T>& a, const OwnFace<T>& F, T te, const T* R, int t,
                                         const ElemInfo& I, const T (&un)[6], const T (&dnn)[6], T (&vt)[6],
                                         T (&gt)[6], T (&gc)[2][3]) {
  constexpr int N3 = N * N * N;
  constexpr TabOff O(N);
  const auto& co = F.co;
  const auto& dA = F.dA;
  const auto& tn = F.tn;
  T uq[N], g0[N], g1[N], g2[N];
  read_line<N, T, d>(R, t, uq);
  constexpr int AS = lds_array_size(N);
  read_line<N, T, d>(R + AS, t, g0);
  read_line<N, T, d>(R + 2 * AS, t, g1);
  read_line<N, T, d>(R + 3 * AS, t, g2);
  const cptr<T> c = fresh(a.tabs);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    T uo = 0, h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T l = c[(s ? O.lg1() : O.lg0()) + m];
      uo += l * uq[m];
      h0 += l * g0[m];
      h1 += l * g1[m];
      h2 += l * g2[m];
    }
    const bool hf = has_nb(I, f);
    const bool neu = !hf && ((a.bcmask >> f) & 1);  // Neumann: no face term
    const T dno = co[s][0] * h0 + co[s][1] * h1 + co[s][2] * h2;
    // interior: [u] = u- - u+, {du/dn}; Dirichlet mirror: u+ = -u-, grad u+ = grad u-
    const T jump = hf ? uo - un[f] : T(2) * uo;
    const T avg = hf ? T(0.5) * (dno + dnn[f]) : dno;
    const T w = neu ? T(0) : dA[s];
    vt[f] = (tau_face(te, tn[s], hf) * jump - avg) * w;
    gt[f] = T(-0.5) * jump * w;
    if constexpr (PRE) {
#pragma unroll
      for (int r = 0; r < 3; ++r) gc[s][r] = co[s][r] * gt[f];
    }
  }
}

// Add the face tests of direction d to the d-lines of the integration
// arrays from the products gc of the own-side metric and gt (no loads).
template <int N, typename T, int d>
__device__ __forceinline__ void inject_pre(const OpArgs<T>& a, const T (&vt)[6], const T (&gc)[2][3], T (&vq)[N],
                                           T (&fx)[N], T (&fy)[N], T (&fz)[N]) {
  constexpr TabOff O(N);
  const cptr<T> c = fresh(a.tabs);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T l = c[(s ? O.lg1() : O.lg0()) + m];
      vq[m] += l * vt[f];
      fx[m] += l * gc[s][0];
      fy[m] += l * gc[s][1];
      fz[m] += l * gc[s][2];
    }
  }
}

// Add the face tests of direction d to the d-lines of the integration
// arrays (vq: test value, fx/fy/fz: test reference gradient).
template <int N, typename T, int d>
__device__ __forceinline__ void inject(const OpArgs<T>& a, const ElemInfo& I, int t, const T (&vt)[6],
                                       const T (&gt)[6], T (&vq)[N], T (&fx)[N], T (&fy)[N], T (&fz)[N]) {
  constexpr TabOff O(N);
  T cd[2][3];
  face_metric<N, T, d, true>(a, I, 0, t, cd[0]);
  face_metric<N, T, d, true>(a, I, 1, t, cd[1]);
  const cptr<T> c = fresh(a.tabs);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int f = 2 * d + s;
    const T c0 = cd[s][0] * gt[f], c1 = cd[s][1] * gt[f], c2 = cd[s][2] * gt[f];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const T l = c[(s ? O.lg1() : O.lg0()) + m];
      vq[m] += l * vt[f];
      fx[m] += l * c0;
      fy[m] += l * c1;
      fz[m] += l * c2;
    }
  }
}

// ------------------------------------------------------------------ affine faces
// Nodal face terms of direction d added to the x-line accumulator vacc.
// With n^T J^{-T} = +-e_d / h_d on both sides and surface weight
// h_a h_b w_a w_b, the flux reduces to the plane term tau [u] - c {du/dn}
// and the normal-derivative term -c/2 [u], each taken through the face mass
// matrix M (x) M.  A: own nodal u; F: LDS scratch of 4 n^2; LT: lane tables;
// Pn, Qn, tn of face f = 2d + s: the neighbour line's end value, its
// normal-derivative combination and the neighbour's penalty (loaded for all
// six faces at once by affine_nb); te: the own penalty.
template <int N, typename T, int d>
__device__ __forceinline__ void affine_faces(const OpArgs<T>& a, const T* A, T* F, const T* LT, bool act, int t,
                                             const ElemInfo& I, T (&vacc)[N], const T (&Pn6)[6],
                                             const T (&Qn6)[6], const T (&tn)[6], T te) {
  constexpr int NT = N * N;
  constexpr int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
  constexpr TabOff O(N);
  const int ta = t % N, tbb = t / N;
  if (act) {
    T line[N];
    read_line<N, T, d>(A, t, line);
    const cptr<T> c = fresh(a.tabs);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * d + s;
      const bool hf = has_nb(I, f);
      const bool neu = !hf && ((a.bcmask >> f) & 1);
      const T Po = line[s * (N - 1)];
      T Qo = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) Qo += c[(s ? O.dl1() : O.dl0()) + m] * line[m];
      const T Pn = Pn6[f], Qn = Qn6[f];
      const T Pj = hf ? Po - Pn : (neu ? T(0) : T(2) * Po);
      const T Qs = hf ? Qo + Qn : (neu ? T(0) : T(2) * Qo);
      const T cdn = (s ? T(1) : T(-1)) / a.h[d];
      F[(2 * s) * NT + t] = tau_face(te, tn[f], hf) * Pj - T(0.5) * cdn * Qs;
      F[(2 * s + 1) * NT + t] = T(-0.5) * cdn * Pj;
    }
  }
  group_sync<op_group_lanes(N)>();
  T Z[4] = {0, 0, 0, 0};
  if (act) {
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
      for (int q = 0; q < N; ++q) Z[cc] += LT[O.M() + ta * N + q] * F[cc * NT + q + N * tbb];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) pin(Z[cc]);
  }
  group_sync<op_group_lanes(N)>();
  if (act)
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) F[cc * NT + t] = Z[cc];
  group_sync<op_group_lanes(N)>();
  T W[4] = {0, 0, 0, 0};
  if (act) {
    const T hab = a.h[da] * a.h[db];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
#pragma unroll
      for (int q = 0; q < N; ++q) W[cc] += LT[O.M() + tbb * N + q] * F[cc * NT + ta + N * q];
      W[cc] *= hab;
      pin(W[cc]);
    }
  }
  group_sync<op_group_lanes(N)>();
  if (act)
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) F[cc * NT + t] = W[cc];
  group_sync<op_group_lanes(N)>();
  // F[(2s) n^2 + node]: plane term at the end node; F[(2s+1) n^2 + node]:
  // weight of l_i'(s) along the normal line.  Add into this lane's x-line.
  if (act) {
    const cptr<T> c = fresh(a.tabs);
    const int j = t % N, l = t / N;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* Pv = F + (2 * s) * NT;
      const T* Qv = F + (2 * s + 1) * NT;
      const int endp = s * (N - 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (d == 0) {
          vacc[i] += (i == endp ? Pv[t] : T(0)) + c[(s ? O.dl1() : O.dl0()) + i] * Qv[t];
        } else if (d == 1) {
          vacc[i] += (j == endp ? Pv[i + N * l] : T(0)) + LT[(s ? O.dl1() : O.dl0()) + j] * Qv[i + N * l];
        } else {
          vacc[i] += (l == endp ? Pv[i + N * j] : T(0)) + LT[(s ? O.dl1() : O.dl0()) + l] * Qv[i + N * j];
        }
      }
    }
  }
  group_sync<op_group_lanes(N)>();
}

// Element of work item `item` = element * nrhs + vector.  With several
// vectors, items are below 2^31 and nrhs <= 64 (both checked at launch), and
// the quotient comes from the host's FP64 1/nrhs instead of an integer
// division: (item + 1/2) / nrhs lies at least 1/(2 nrhs) >= 2^-7 from an
// integer, and the two rounded FP64 operations move it by less than 2^-21,
// so truncation gives the exact quotient.
template <typename T>
__device__ __forceinline__ int64_t item_elem(const OpArgs<T>& a, int64_t item) {
  if (a.nrhs == 1) return item;
  return (int64_t)exact_div((unsigned)item, a.inv_nrhs);
}

// Offset of the first value of work item `item` (element x vector) in the
// vectors of a launch.
template <int N, typename T>
__device__ __forceinline__ int64_t item_offset(const OpArgs<T>& a, int64_t item) {
  constexpr int N3 = N * N * N;
  if (a.nrhs == 1) return item * N3;
  const int64_t el = item_elem(a, item);
  return (item - el * a.nrhs) * a.ld + el * N3;
}
// Work items of a launch in linear order from it0: how many are left
// (the group takes at most its EW of them).
template <typename T>
__device__ __forceinline__ int group_count(const OpArgs<T>& a, int64_t it0) {
  const int64_t left = a.nel * a.nrhs - it0;
  return left <= 0 ? 0 : (left > 1024 ? 1024 : (int)left);
}

// ------------------------------------------------------------------ operator
// Lane tables (the per-lane part of op_tables()) into a group's LDS (GL
// lanes): loads first, one round trip.
template <typename T, int LTN, int GL>
__device__ __forceinline__ void load_lane_tables(const T* tabs, T* LT) {
  const int lane = threadIdx.x & (GL - 1);
  constexpr int KL = (LTN + GL - 1) / GL;
  T lt[KL];
#pragma unroll
  for (int i = 0; i < KL; ++i) lt[i] = tabs[lane + GL * i < LTN ? lane + GL * i : 0];
  // all loads are issued before the first store (otherwise the compiler
  // sinks the last ones past the stores: a second round trip)
#pragma unroll
  for (int i = 0; i < KL; ++i) pin(lt[i]);
#pragma unroll
  for (int i = 0; i < KL; ++i)
    if (lane + GL * i < LTN) LT[lane + GL * i] = lt[i];
}

// One group's share of a launch: the work items it0 .. it0 + nv - 1 (at
// most EW of them; nv <= 0: none).  Work items are (element, vector) pairs,
// vector fastest, so with several vectors the slots of a group share one
// element's geometry (the same cache lines); slots past nv are idle lanes.
// W0 is the group's LDS region: EW * PER values, then the lane tables
// (filled by the caller).  Phases are separated by group_sync().  Each
// phase is one `if (act)` block whose global loads are issued together at
// its start (clamped addresses, no per-face branches), so a phase costs one
// memory round trip.  Returns the wavefront's sum of u.(A u) in OP_DOT
// mode, 0 otherwise.  IN_LOOP (kernels that loop over tiles): the lane
// index is made opaque so that lane arithmetic is redone per call instead
// of being hoisted out of the loop, where it would stay live throughout.
template <int N, typename T, bool CURVED, bool FE, int MODE, bool IN_LOOP = false>
__device__ __forceinline__ double op_items(const OpArgs<T>& a, const int64_t it0, const int nv, T* const W0) {
  using C = Cfg<N, CURVED, FE>;
  constexpr int NT = C::NT, N3 = C::N3, EW = C::EW, PER = C::PER, GL = C::GL;
  constexpr TabOff O(N);
  int lane = threadIdx.x & (GL - 1);
  if constexpr (IN_LOOP) asm volatile("" : "+v"(lane));
  const int le = lane / NT, t = lane - le * NT;
  // one element per wavefront (n = 8): the item, its element and all its
  // index arithmetic are the same on every lane and stay in scalar registers
  const int64_t it = EW == 1 ? it0 : it0 + le;
  const int64_t e = item_elem(a, it);
  const T* const ub = a.u + (a.nrhs == 1 ? 0 : (it - e * a.nrhs) * a.ld);  // this lane's vector
  const bool act = (le < EW) && (le < nv);
  T* const R = W0 + (le < EW ? le : 0) * PER;
  T* const LT = W0 + EW * PER;
  const ElemInfo I = elem_info(a, e);
  const int nload = (nv <= 0 ? 0 : (nv < EW ? nv : EW)) * N3;
  const int ta = t % N, tbb = t / N;

  // ---- neighbour traces (curved DG), before the own data occupies LDS.
  // For n >= 7 and FP64 n = 5 the own values are loaded into registers
  // with the neighbour data (one round trip for both) and go to LDS once the
  // neighbour phase is done; elsewhere the registers would cost a wavefront
  // per SIMD.  FP64 n = 6 with workgroup groups holds 6 values per lane
  // (7 elements on 256 lanes), which spilled 11 registers and was 2-3%
  // slower than loading them after the neighbour phase.
  constexpr int OWN_PER_LANE = (EW * N3 + GL - 1) / GL;
  constexpr bool early_own =
      CURVED && !FE && (N >= 7 || (N == 5 && sizeof(T) == 8) || (N == 6 && sizeof(T) == 8 && GL == 64));
  [[maybe_unused]] T own[OWN_PER_LANE];
  T un[6], dnn[6];
  if constexpr (CURVED && !FE) {
    // neighbour-side face metric: for n = 5, 7, 8 loaded with the
    // neighbour lines (one round trip less, 1-2% faster); for the other
    // degrees the registers it holds across the two LDS sweeps below would
    // cost a wavefront per SIMD, so it is loaded after them
    constexpr bool early_cn = N == 5 || N >= 7;
    T cn[6][3];
    if constexpr (early_own) {
#pragma unroll
      for (int j = 0; j < OWN_PER_LANE; ++j) {
        const int idx = lane + GL * j;
        const int li = EW == 1 ? 0 : idx / N3;
        own[j] = idx < nload ? a.u[item_offset<N>(a, it0 + li) + (idx - li * N3)] : T(0);
      }
    }
    {  // neighbour lines of all six faces: end value P, normal derivative Q
      T nl[6][N];
      load_nb_lines<N, T, 0>(a, ub, I, t, nl[0], nl[1]);
      load_nb_lines<N, T, 1>(a, ub, I, t, nl[2], nl[3]);
      load_nb_lines<N, T, 2>(a, ub, I, t, nl[4], nl[5]);
      if constexpr (early_cn) nb_face_metric<N, T>(a, I, t, cn);
      const cptr<T> c = fresh(a.tabs);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int s = f & 1;
        T Q = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) Q += c[(s ? O.dl0() : O.dl1()) + m] * nl[f][m];
        if (act) {
          R[(2 * f) * NT + t] = s ? nl[f][0] : nl[f][N - 1];
          R[(2 * f + 1) * NT + t] = Q;
        }
      }
    }
    group_sync<GL>();
    T X[18];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      X[3 * f] = X[3 * f + 1] = X[3 * f + 2] = 0;
      if (act)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          const T sv = LT[O.S() + ta * N + q], sp = LT[O.Sp() + ta * N + q];
          const T p = R[(2 * f) * NT + q + N * tbb], qq = R[(2 * f + 1) * NT + q + N * tbb];
          X[3 * f] += sv * p;
          X[3 * f + 1] += sp * p;
          X[3 * f + 2] += sv * qq;
        }
    }
    group_sync<GL>();
    if (act)
#pragma unroll
      for (int cc = 0; cc < 18; ++cc) R[cc * NT + t] = X[cc];
    group_sync<GL>();
#pragma unroll
    for (int f = 0; f < 6; ++f) un[f] = dnn[f] = 0;
    if (act) {
      if constexpr (!early_cn) nb_face_metric<N, T>(a, I, t, cn);
      nb_finish<N, T, 0>(R, LT, t, I, cn, un, dnn);
      nb_finish<N, T, 1>(R, LT, t, I, cn, un, dnn);
      nb_finish<N, T, 2>(R, LT, t, I, cn, un, dnn);
    }
    group_sync<GL>();
  }


  // affine faces: the neighbour lines of all six faces reduced at once to
  // their end value and normal-derivative combination, with the penalties
  // (one memory round trip, together with the own values below, instead of
  // one per direction)
  [[maybe_unused]] T aPn[6], aQn[6], atn[6];
  [[maybe_unused]] T ate = 0;
  if constexpr (!CURVED && !FE) {
    if (act) {
      T nl[6][N];
      load_nb_lines<N, T, 0>(a, ub, I, t, nl[0], nl[1]);
      load_nb_lines<N, T, 1>(a, ub, I, t, nl[2], nl[3]);
      load_nb_lines<N, T, 2>(a, ub, I, t, nl[4], nl[5]);
      ate = a.tau[I.e];
      atn[0] = a.tau[nb_elem<0>(a, I, 0)];
      atn[1] = a.tau[nb_elem<0>(a, I, 1)];
      atn[2] = a.tau[nb_elem<1>(a, I, 0)];
      atn[3] = a.tau[nb_elem<1>(a, I, 1)];
      atn[4] = a.tau[nb_elem<2>(a, I, 0)];
      atn[5] = a.tau[nb_elem<2>(a, I, 1)];
      const cptr<T> c = fresh(a.tabs);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int s = f & 1;
        T Q = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) Q += c[(s ? O.dl0() : O.dl1()) + m] * nl[f][m];
        aQn[f] = Q;
        aPn[f] = s ? nl[f][0] : nl[f][N - 1];
      }
    }
  }

  // own-side face data: for n = 5 and 8 each direction's is loaded a phase
  // ahead of its use, those of the x faces in the phase that moves the own
  // values to LDS (1-2% faster; for n = 3, 4, 6 the registers cost a
  // wavefront per SIMD); otherwise in the phase that uses it
  constexpr bool pf_faces = N == 5 || N == 8;
  [[maybe_unused]] OwnFace<T> F0, F1, F2;
  [[maybe_unused]] T te = 0;
  if constexpr (CURVED && !FE && pf_faces) {
    F0 = load_own_face<N, T, 0>(a, I, t);
    te = a.tau[I.e];
  }

  // ---- own element data into LDS (coalesced per group)
  if constexpr (early_own) {
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      if (idx < nload) {
        const int li = EW == 1 ? 0 : idx / N3;
        W0[li * PER + vpos_of<N>(idx - li * N3)] = own[j];
        if constexpr (keeps_input<N, T, CURVED, FE, MODE>()) LT[C::LT + idx] = own[j];
      }
    }
  } else if constexpr (!FE) {
    // all of the lane's loads first, then the LDS stores: one memory round
    // trip (a load-store loop waits for each load in turn)
    T v[OWN_PER_LANE];
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      const int li = EW == 1 ? 0 : idx / N3;
      v[j] = idx < nload ? a.u[item_offset<N>(a, it0 + li) + (idx - li * N3)] : T(0);
    }
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      if (idx < nload) {
        const int li = EW == 1 ? 0 : idx / N3;
        W0[li * PER + vpos_of<N>(idx - li * N3)] = v[j];
        if constexpr (keeps_input<N, T, CURVED, FE, MODE>()) LT[C::LT + idx] = v[j];
      }
    }
  } else {
    // continuous FE levels: work item = (element, vector), vector fastest,
    // vector r of the input r * ld values after the first; element and node
    // indices fit in 32 bits (the level's node count is checked on the host).
    // All of the lane's gathers first, then the LDS stores (one round trip).
    constexpr int k = N - 1;
    const int Mx = a.Nx * k + 1, My = a.Ny * k + 1, Mz = a.Nz * k + 1;
    T v[OWN_PER_LANE];
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      const int li = EW == 1 ? 0 : idx / N3, p = idx - li * N3;
      const int64_t item = it0 + li;
      const int64_t elv = item_elem(a, item);
      const T* const uv = a.u + (a.nrhs == 1 ? 0 : (item - elv * a.nrhs) * a.ld);
      const unsigned ee = (unsigned)elv, rr = exact_div(ee, a.inv_nx), ez = exact_div(rr, a.inv_ny);
      const int gx = (int)(ee - rr * a.Nx) * k + p % N;
      const int gy = (int)(rr - ez * a.Ny) * k + (p / N) % N;
      const int gz = (int)ez * k + p / NT;
      const int m = a.bcmask;
      const bool fixed = (gx == 0 && !(m & 1)) || (gx == Mx - 1 && !(m & 2)) || (gy == 0 && !(m & 4)) ||
                         (gy == My - 1 && !(m & 8)) || (gz == 0 && !(m & 16)) || (gz == Mz - 1 && !(m & 32));
      v[j] = (idx < nload && !fixed) ? uv[gx + (int64_t)Mx * (gy + (int64_t)My * gz)] : T(0);
    }
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      if (idx < nload) {
        const int li = EW == 1 ? 0 : idx / N3;
        W0[li * PER + vpos_of<N>(idx - li * N3)] = v[j];
      }
    }
  }
  group_sync<GL>();

  T* const A = R;
  T* const B = R + C::AS;
  T* const Cc = R + 2 * C::AS;
  T v[N];

  if constexpr (!CURVED) {
    // ---- affine: faces in nodal space, cell as sum_d c_d K_d (x) M (x) M
    T vacc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) vacc[i] = 0;
    if constexpr (!FE) {
      affine_faces<N, T, 0>(a, A, B, LT, act, t, I, vacc, aPn, aQn, atn, ate);
      affine_faces<N, T, 1>(a, A, B, LT, act, t, I, vacc, aPn, aQn, atn, ate);
      affine_faces<N, T, 2>(a, A, B, LT, act, t, I, vacc, aPn, aQn, atn, ate);
    }
    const T cx = a.h[1] * a.h[2] / a.h[0], cy = a.h[0] * a.h[2] / a.h[1], cz = a.h[0] * a.h[1] / a.h[2];
    if (act) {  // z: p = M u, q = K u
      const cptr<T> c = fresh(a.tabs);
      T x[N], p[N], q[N];
      read_line<N, T, 2>(A, t, x);
      eo_apply<N, T, 1>(c + O.eo(EO_M), x, p);
      eo_apply<N, T, 1>(c + O.eo(EO_K), x, q);
      write_line<N, T, 2>(B, t, p);
      write_line<N, T, 2>(Cc, t, q);
    }
    group_sync<GL>();
    if (act) {  // y: r = M p, s = cy K p + cz M q
      const cptr<T> c = fresh(a.tabs);
      T p[N], q[N], r[N], s1[N], s2[N];
      read_line<N, T, 1>(B, t, p);
      read_line<N, T, 1>(Cc, t, q);
      eo_apply<N, T, 1>(c + O.eo(EO_M), p, r);
      eo_apply<N, T, 1>(c + O.eo(EO_K), p, s1);
      eo_apply<N, T, 1>(c + O.eo(EO_M), q, s2);
#pragma unroll
      for (int m = 0; m < N; ++m) s1[m] = cy * s1[m] + cz * s2[m];
      write_line<N, T, 1>(B, t, r);
      write_line<N, T, 1>(Cc, t, s1);
    }
    group_sync<GL>();
    if (act) {  // x: v = cx K r + M s
      const cptr<T> c = fresh(a.tabs);
      T r[N], s[N], v1[N], v2[N];
      read_line<N, T, 0>(B, t, r);
      read_line<N, T, 0>(Cc, t, s);
      eo_apply<N, T, 1>(c + O.eo(EO_K), r, v1);
      eo_apply<N, T, 1>(c + O.eo(EO_M), s, v2);
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] = cx * v1[m] + v2[m] + vacc[m];
    }
  } else {
    // FE levels have no face data: the z-derivative is formed from the
    // lane's own z-line in the metric phase, and the z-flux then takes the
    // place of the Gauss-point values (three arrays instead of four)
    T* const Dg = FE ? A : R + 3 * C::AS;
    // ---- curved: interpolation to Gauss points, x then y then z
    if (act) {
      const cptr<T> c = fresh(a.tabs);
      T x[N], y[N];
      read_line<N, T, 0>(A, t, x);
      eo_apply<N, T, 1>(c + O.eo(EO_S), x, y);
      write_line<N, T, 0>(A, t, y);
    }
    group_sync<GL>();
    if (act) {
      const cptr<T> c = fresh(a.tabs);
      T x[N], y[N];
      read_line<N, T, 1>(A, t, x);
      eo_apply<N, T, 1>(c + O.eo(EO_S), x, y);
      write_line<N, T, 1>(A, t, y);
    }
    group_sync<GL>();
    if (act) {
      const cptr<T> c = fresh(a.tabs);
      T x[N], uq[N];
      [[maybe_unused]] T gz[N];
      read_line<N, T, 2>(A, t, x);
      eo_apply<N, T, 1>(c + O.eo(EO_S), x, uq);
      write_line<N, T, 2>(A, t, uq);
      if constexpr (!FE) {
        eo_apply<N, T, -1>(c + O.eo(EO_D), uq, gz);
        write_line<N, T, 2>(Dg, t, gz);
      }
    }
    group_sync<GL>();
    if (act) {  // collocation derivatives in x (-> B) and y (-> Cc)
      const cptr<T> c = fresh(a.tabs);
      T x[N], y[N];
      read_line<N, T, 0>(A, t, x);
      eo_apply<N, T, -1>(c + O.eo(EO_D), x, y);
      write_line<N, T, 0>(B, t, y);
      read_line<N, T, 1>(A, t, x);
      eo_apply<N, T, -1>(c + O.eo(EO_D), x, y);
      write_line<N, T, 1>(Cc, t, y);
    }
    group_sync<GL>();
    // ---- face fluxes (DG): own traces by extrapolation
    // x- and y-face tests: the products of the own-side metric with gt are
    // formed in the flux phase (the metric is in registers there), so the
    // test phases need no second load of it.  z faces: their tests join the
    // metric phase, whose loads are one round trip anyway; the products save
    // six loads there, and for n = 4, 6 they cost a wavefront per SIMD
    // (FP32, n = 4) or spill (FP64, n = 6)
    constexpr bool pre_gc_z = N == 5 || N >= 7;
    T vt[6], gt[6];
    T gc0[2][3], gc1[2][3];
    [[maybe_unused]] T gc2[2][3];
    if constexpr (!FE) {
#pragma unroll
      for (int f = 0; f < 6; ++f) vt[f] = gt[f] = 0;
      // one direction per block (the fences keep the blocks from being
      // merged, which would put all three directions' data in flight)
      if constexpr (pf_faces) {
        F1 = load_own_face<N, T, 1>(a, I, t);
      } else {
        F0 = load_own_face<N, T, 0>(a, I, t);
        te = a.tau[I.e];
      }
      if (act) own_flux<N, T, 0, true>(a, F0, te, R, t, I, un, dnn, vt, gt, gc0);
      group_sync<GL>();
      if constexpr (pf_faces)
        F2 = load_own_face<N, T, 2>(a, I, t);
      else
        F1 = load_own_face<N, T, 1>(a, I, t);
      if (act) own_flux<N, T, 1, true>(a, F1, te, R, t, I, un, dnn, vt, gt, gc1);
      group_sync<GL>();
      if constexpr (!pf_faces) F2 = load_own_face<N, T, 2>(a, I, t);
      if (act) own_flux<N, T, 2, pre_gc_z>(a, F2, te, R, t, I, un, dnn, vt, gt, gc2);
      group_sync<GL>();
    }
    // ---- quadrature-point operator on z-lines, z-face tests
    if (act) {
      T vq[N], fx[N], fy[N], fz[N];
      [[maybe_unused]] T gzl[N];
      if constexpr (FE) {  // z-derivative of the lane's own z-line
        const cptr<T> c = fresh(a.tabs);
        T x[N];
        read_line<N, T, 2>(A, t, x);
        eo_apply<N, T, -1>(c + O.eo(EO_D), x, gzl);
      }
      const T* G = a.metric + e * 6 * N3 + t;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int o = sidx<N, 2>(t, m);
        const T gx = B[o], gy = Cc[o];
        T g3;
        if constexpr (FE) g3 = gzl[m];
        else g3 = Dg[o];
        const T* Gm = G + NT * m;
        // stored order 00, 11, 22, 01, 02, 12
        const T g00 = Gm[0], g11 = Gm[N3], g22 = Gm[2 * N3];
        const T g01 = Gm[3 * N3], g02 = Gm[4 * N3], g12 = Gm[5 * N3];
        fx[m] = g00 * gx + g01 * gy + g02 * g3;
        fy[m] = g01 * gx + g11 * gy + g12 * g3;
        fz[m] = g02 * gx + g12 * gy + g22 * g3;
        vq[m] = 0;
      }
      if constexpr (!FE) {
        if constexpr (pre_gc_z)
          inject_pre<N, T, 2>(a, vt, gc2, vq, fx, fy, fz);
        else
          inject<N, T, 2>(a, I, t, vt, gt, vq, fx, fy, fz);
      }
      if constexpr (!FE) write_line<N, T, 2>(A, t, vq);
      write_line<N, T, 2>(B, t, fx);
      write_line<N, T, 2>(Cc, t, fy);
      write_line<N, T, 2>(Dg, t, fz);
    }
    group_sync<GL>();
    if constexpr (!FE) {  // x-face tests along x-lines
      if (act) {
        T vq[N], fx[N], fy[N], fz[N];
        read_line<N, T, 0>(A, t, vq);
        read_line<N, T, 0>(B, t, fx);
        read_line<N, T, 0>(Cc, t, fy);
        read_line<N, T, 0>(Dg, t, fz);
        inject_pre<N, T, 0>(a, vt, gc0, vq, fx, fy, fz);
        write_line<N, T, 0>(A, t, vq);
        write_line<N, T, 0>(B, t, fx);
        write_line<N, T, 0>(Cc, t, fy);
        write_line<N, T, 0>(Dg, t, fz);
      }
      group_sync<GL>();
    }
    if (act) {  // y-face tests, then integration in y
      T fx[N], fy[N], fz[N], ay[N], by[N], cy[N], w2[N];
      read_line<N, T, 1>(B, t, fx);
      read_line<N, T, 1>(Cc, t, fy);
      read_line<N, T, 1>(Dg, t, fz);
      if constexpr (!FE) {
        T vq[N];
        read_line<N, T, 1>(A, t, vq);
        inject_pre<N, T, 1>(a, vt, gc1, vq, fx, fy, fz);
        const cptr<T> c = fresh(a.tabs);
        eo_apply<N, T, 1>(c + O.eo(EO_ST), vq, cy);
      }
      const cptr<T> c = fresh(a.tabs);
      eo_apply<N, T, 1>(c + O.eo(EO_ST), fx, ay);
      eo_apply<N, T, 1>(c + O.eo(EO_ST), fz, by);
      eo_apply<N, T, -1>(c + O.eo(EO_SPT), fy, w2);
#pragma unroll
      for (int m = 0; m < N; ++m) cy[m] = FE ? w2[m] : cy[m] + w2[m];
      write_line<N, T, 1>(A, t, ay);
      write_line<N, T, 1>(B, t, by);
      write_line<N, T, 1>(Cc, t, cy);
    }
    group_sync<GL>();
    if (act) {  // integration in z
      const cptr<T> c = fresh(a.tabs);
      T ay[N], by[N], cy[N], az[N], bz[N], w2[N];
      read_line<N, T, 2>(A, t, ay);
      read_line<N, T, 2>(B, t, by);
      read_line<N, T, 2>(Cc, t, cy);
      eo_apply<N, T, 1>(c + O.eo(EO_ST), ay, az);
      eo_apply<N, T, 1>(c + O.eo(EO_ST), cy, w2);
      eo_apply<N, T, -1>(c + O.eo(EO_SPT), by, bz);
#pragma unroll
      for (int m = 0; m < N; ++m) bz[m] += w2[m];
      write_line<N, T, 2>(A, t, az);
      write_line<N, T, 2>(B, t, bz);
    }
    group_sync<GL>();
    if (act) {  // integration in x
      const cptr<T> c = fresh(a.tabs);
      T az[N], bz[N], w2[N];
      read_line<N, T, 0>(A, t, az);
      read_line<N, T, 0>(B, t, bz);
      eo_apply<N, T, -1>(c + O.eo(EO_SPT), az, v);
      eo_apply<N, T, 1>(c + O.eo(EO_ST), bz, w2);
#pragma unroll
      for (int m = 0; m < N; ++m) v[m] += w2[m];
    }
  }
  group_sync<GL>();
  if (act) write_line<N, T, 0>(A, t, v);
  group_sync<GL>();

  // ---- coalesced epilogue over the group's elements.  The vectors it reads
  // (residual, Chebyshev update, u.(A u)) are loaded for all of the lane's
  // values first, then combined and stored: one memory round trip (a
  // load-store loop waits for each value's loads in turn)
  double acc = 0.0;
  constexpr bool KI = keeps_input<N, T, CURVED, FE, MODE>();
  constexpr bool LX = !FE && (MODE == OP_CHEB || MODE == OP_DOT) && !KI;  // loads u
  constexpr bool LB = !FE && (MODE == OP_RESID || MODE == OP_CHEB);      // loads b
  constexpr bool LC = !FE && MODE == OP_CHEB;                            // loads x_old, dinv
  // offsets of value idx: g in the launch's vectors, gv inside one vector
  auto offsets = [&](int idx, int64_t& g, int64_t& gv) {
    const int li = EW == 1 ? 0 : idx / N3;
    const int64_t item = it0 + li;
    const int64_t el = item_elem(a, item);
    gv = el * N3 + (idx - li * N3);
    // FE levels write element-local results, n_el n^3 values per vector
    g = gv + (a.nrhs == 1 ? 0 : (item - el * a.nrhs) * (FE ? a.nel * N3 : a.ld));
  };
  [[maybe_unused]] T ex[LX ? OWN_PER_LANE : 1], eb[LB ? OWN_PER_LANE : 1], eo[LC ? OWN_PER_LANE : 1],
      ed[LC ? OWN_PER_LANE : 1];
  if constexpr (LX || LB || LC) {
    const T* const xop = a.xold ? a.xold : a.u;  // NULL x_old: loaded from u, used as 0
#pragma unroll
    for (int j = 0; j < OWN_PER_LANE; ++j) {
      const int idx = lane + GL * j;
      if (idx < nload) {
        int64_t g, gv;
        offsets(idx, g, gv);
        if constexpr (LX) ex[j] = a.u[g];
        if constexpr (LB) eb[j] = a.b[g];
        if constexpr (LC) {
          eo[j] = xop[g];
          ed[j] = a.dinv[gv];
        }
      }
    }
  }
  if constexpr (FE || MODE == OP_APPLY) {  // stores only
    for (int idx = lane; idx < nload; idx += GL) {
      const int li = EW == 1 ? 0 : idx / N3;
      int64_t g, gv;
      offsets(idx, g, gv);
      a.out[g] = W0[li * PER + vpos_of<N>(idx - li * N3)];
    }
    return acc;
  }
#pragma unroll
  for (int j = 0; j < OWN_PER_LANE; ++j) {
    const int idx = lane + GL * j;
    if (idx < nload) {
      const int li = EW == 1 ? 0 : idx / N3;
      const T val = W0[li * PER + vpos_of<N>(idx - li * N3)];
      int64_t g, gv;
      offsets(idx, g, gv);
      if constexpr (FE || MODE == OP_APPLY) {
        a.out[g] = val;
      } else if constexpr (MODE == OP_RESID) {
        a.out[g] = eb[j] - val;
      } else if constexpr (MODE == OP_CHEB) {
        T x;
        if constexpr (KI) x = LT[C::LT + idx];  // kept in LDS
        else x = ex[j];
        const T xo = a.xold ? eo[j] : T(0);  // NULL: x_old = 0 (second step from a zero start)
        a.out[g] = x + a.sigma * (x - xo) + a.theta * ed[j] * (eb[j] - val);
      } else {
        a.out[g] = val;
        if constexpr (KI) acc += (double)LT[C::LT + idx] * (double)val;
        else acc += (double)ex[j] * (double)val;
      }
    }
  }
  if constexpr (!FE && MODE == OP_DOT)
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  return acc;
}

// ------------------------------------------------------------------ multi mesh
// Device view of a multi-mesh launch (MultiLaunch): tiles of q workgroup
// chunks of one mesh each.
template <typename T>
struct MultiArgs {
  const MeshEntry<T>* table;
  int count, q;
  const int64_t* xcd;
};

template <typename T>
inline MultiArgs<T> multi_args(const MultiLaunch& L) {
  MultiArgs<T> m;
  m.table = (const MeshEntry<T>*)L.table;
  m.count = L.count;
  m.q = L.q;
  m.xcd = L.xcd;
  return m;
}

// Index of the mesh holding `tile` (tile0 ascending; uniform loop).
template <typename T>
__device__ __forceinline__ int find_mesh(cptr<MeshEntry<T>> tab, int count, int64_t tile) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tab[mid].tile0 <= tile) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The chunks of one tile of mesh E; the lane tables of E's degree are in
// the group's LDS.  The mesh's arguments (vector pointers resolved for
// this launch) are read in place from the constant table where they are
// used, as kernel arguments are, instead of being held in registers.
template <int N, typename T, bool CURVED, int MODE>
__device__ __forceinline__ void multi_tile(const MultiArgs<T>& m, cptr<MeshEntry<T>> E, int64_t tile, T* W0) {
  using C = Cfg<N, CURVED, false>;
  const int64_t c0 = (tile - E->tile0) * m.q;
  const int64_t c1 = c0 + m.q < E->chunks ? c0 + m.q : E->chunks;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / C::GL);  // group-uniform (scalar)
  for (int64_t c = c0; c < c1; ++c) {
    group_sync<C::GL>();  // the previous chunk's LDS reads come first
    // an opaque copy of the entry pointer per chunk: the argument loads are
    // not hoisted out of the loop (where they would stay live throughout)
    cptr<MeshEntry<T>> Ec = E;
    asm volatile("" : "+s"(Ec)::"memory");
    const OpArgs<T>& a = *(const OpArgs<T>*)&Ec->a;
    const int64_t it0 = c * C::EB + (int64_t)grp * C::EW;
    op_items<N, T, CURVED, false, MODE, true>(a, it0, group_count(a, it0), W0);
  }
}

}  // namespace hmg
