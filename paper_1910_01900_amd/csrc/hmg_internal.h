// Internal declarations shared by the host setup, the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hmg.h"

namespace hmg {

constexpr int kMaxN = 8;  // n = k + 1, k = 1..7

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define HMG_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::hmg::fail(HMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
int check_launch(const char* what);
// HMG_ERR_INVALID unless p is non-null and 256-byte aligned
int check_ptr(const void* p, const char* what);
#define TRY(x)               \
  do {                       \
    int rc_ = (x);           \
    if (rc_ < 0) return rc_; \
  } while (0)
// Classical Chebyshev iteration coefficients on [lof, hif] * lmax (step j:
// x_{j+1} = x_j + sig[j] (x_j - x_{j-1}) + th[j] D^{-1} (b - A x_j); sig[0] = 0).
void cheb_coeffs(int ns, double lmax, double lof, double hif, std::vector<double>& sig,
                 std::vector<double>& th);

// ---------------------------------------------------------------- 1-D bases
// Sec. 2: Lagrange basis on the k+1 GLL nodes of [0,1], Gauss rule with k+1
// points.  All tables are row-major [q][i].
struct Basis1D {
  int k = 0, n = 0;
  std::vector<double> gll, gz, gw;  // GLL nodes, Gauss points, Gauss weights
  std::vector<double> S;            // S[q][i]  = l_i(z_q)
  std::vector<double> Sp;           // Sp[q][i] = l_i'(z_q)
  std::vector<double> D;            // D[q][r]  = derivative of the Gauss Lagrange basis r at z_q
  std::vector<double> M;            // M[i][j]  = sum_q w_q l_i(z_q) l_j(z_q) (1-D mass)
  std::vector<double> K;            // K[i][j]  = sum_q w_q l_i'(z_q) l_j'(z_q) (1-D stiffness)
  std::vector<double> dl0, dl1;     // l_i'(0), l_i'(1)
  std::vector<double> lg0, lg1;     // Gauss-point Lagrange basis at 0 and 1
};
Basis1D make_basis(int k);
std::vector<double> gll_nodes(int k);
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
// V[q][i] = l_i(x_q), Dv[q][i] = l_i'(x_q) for the Lagrange basis of `nodes`.
void lagrange(const std::vector<double>& nodes, const std::vector<double>& x,
              std::vector<double>* V, std::vector<double>* Dv);

// Operator tables in device memory (level precision), built by op_tables():
//   [S, Sp, M]            n x n row-major, read per lane (face sweeps)
//   [l'(0), l'(1)]        GLL basis derivatives at the element ends
//   [lg(0), lg(1)]        Gauss-point Lagrange basis at the element ends
//   even-odd packed S, S^T, Sp^T, D, M, K (eo_count(n) values each)
// Even-odd packing of an n x n matrix A with A[n-1-q][n-1-i] = sig A[q][i]
// (h = n/2): E[q][i] = (A[q][i] + A[q][n-1-i])/2, O[q][i] = (A[q][i] -
// A[q][n-1-i])/2 for q, i < h; for odd n also A[q][h] (q < h), the middle
// row A[h][i] (i < h) and A[h][h].  Then with x_e = x_i + x_{n-1-i},
// x_o = x_i - x_{n-1-i}: y_q = E x_e + O x_o (+ A[q][h] x_h) and
// y_{n-1-q} = sig (E x_e - O x_o (+ A[q][h] x_h)).
constexpr int eo_count(int n) { return 2 * (n / 2) * (n / 2) + ((n & 1) ? 2 * (n / 2) + 1 : 0); }
struct TabOff {
  int n, nt, c;
  constexpr TabOff(int n_) : n(n_), nt(n_ * n_), c(eo_count(n_)) {}
  constexpr int S() const { return 0; }
  constexpr int Sp() const { return nt; }
  constexpr int M() const { return 2 * nt; }
  constexpr int dl0() const { return 3 * nt; }
  constexpr int dl1() const { return 3 * nt + n; }
  constexpr int lane_size() const { return 3 * nt + 2 * n; }  // part read per lane
  constexpr int lg0() const { return 3 * nt + 2 * n; }
  constexpr int lg1() const { return 3 * nt + 3 * n; }
  constexpr int eo(int j) const { return 3 * nt + 4 * n + j * c; }  // 0 S, 1 S^T, 2 Sp^T, 3 D, 4 M, 5 K
  constexpr int size() const { return eo(6); }
};
enum EoTab { EO_S = 0, EO_ST = 1, EO_SPT = 2, EO_D = 3, EO_M = 4, EO_K = 5 };
std::vector<double> op_tables(const Basis1D& b);

// ---------------------------------------------------------------- mesh / geometry
struct Mesh {
  int N[3];
  double lo[3], hi[3];
  int k;
  bool curved;
  double amp;
  int waves;
  int mapdeg = 3;  // 3: Q3 interpolant of the deformation; 0: the deformation itself
  uint8_t bc[6];
  double ip;
  std::vector<double> tau_scale;  // empty = all ones
  int64_t n_el() const { return (int64_t)N[0] * N[1] * N[2]; }
  double h(int d) const { return (hi[d] - lo[d]) / N[d]; }
  int bcmask() const {  // bit (2d+s) set <=> Neumann
    int m = 0;
    for (int f = 0; f < 6; ++f)
      if (bc[f]) m |= 1 << f;
    return m;
  }
};

// Host geometry of a level (double precision, uploaded in the level precision).
//  metric  [e][6][n^3]: w_q |det J| J^{-1} J^{-T} as (00, 11, 22, 01, 02, 12)
//  face[d] [f][7][n^2]: f = p + (N_d+1)*(ea + N_a*eb); comps 0..2 = n^T J_L^{-T},
//          3..5 = n^T J_R^{-T}, 6 = surface weight; n points from L to R.
//  tau     [e]
struct Geometry {
  std::vector<double> metric;
  std::vector<double> face[3];
  std::vector<double> tau;
};
int build_geometry(const Mesh& m, const Basis1D& b, Geometry& g, bool faces);  // curved or affine
// Physical point and Jacobian at reference point xi of element e (Q3 map).
void map_point(const Mesh& m, int64_t e, const double xi[3], double x[3], double J[9]);
int rhs_sine_host(const Mesh& m, const Basis1D& b, const Geometry& g, double freq,
                  std::vector<double>& out);
// diag(A) of a DG or FE level (setup, host)
int diag_host(const Mesh& m, const Basis1D& b, const Geometry& g, int space,
              std::vector<double>& out);

// ---------------------------------------------------------------- level handle
}  // namespace hmg

struct hmg_level {
  hmg::Mesh mesh;
  int space = HMG_DG;
  int prec = HMG_F64;
  int k = 1, n = 2;
  int64_t n_el = 0, n_dofs = 0, n_dg = 0;  // n_dg = n_el * n^3
  hmg::Basis1D basis;
  hmg::Geometry geom;  // host copy, released after bind
  std::vector<double> diag_h;  // diag(A), computed during create
  // workspace layout (byte offsets) and bound pointers
  size_t ws_bytes = 0;
  size_t off_metric = 0, off_face[3] = {0, 0, 0}, off_tau = 0, off_diag = 0, off_dinv = 0, off_tmp = 0,
         off_scratch = 0, off_part = 0, off_scal = 0, off_tabs = 0;
  char* ws = nullptr;
  bool bound = false;
  size_t elem_size() const { return prec == HMG_F64 ? 8 : 4; }
  void* metric() const { return ws + off_metric; }
  void* face(int d) const { return ws + off_face[d]; }
  void* tau() const { return ws + off_tau; }
  void* diag() const { return ws + off_diag; }  // diag(A), level precision
  void* dinv() const { return ws + off_dinv; }
  void* tmp(int i) const { return ws + off_tmp + (size_t)i * vec_bytes(); }
  void* scratch() const { return ws + off_scratch; }  // DG-layout buffer (FE levels)
  double* partials() const { return (double*)(ws + off_part); }
  double* scal() const { return (double*)(ws + off_scal); }
  void* tabs() const { return ws + off_tabs; }  // op_tables(basis), level precision
  size_t vec_bytes() const { return (size_t)n_dofs * elem_size(); }
};

namespace hmg {

constexpr int kPartials = 1024;  // max blocks of a reduction
constexpr int kTmpVecs = 4;      // level temporaries (Chebyshev, lambda_max)
constexpr int kMaxRhs = 64;      // vectors per batched launch
constexpr int kPartialsB = 256;  // max blocks per vector of a several-vector reduction

// ---------------------------------------------------------------- kernel launchers
enum OpMode { OP_APPLY = 0, OP_RESID = 1, OP_CHEB = 2, OP_DOT = 3 };

// Arguments of the operator kernels (one mesh).
template <typename T>
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
  const T* tabs;  // op_tables() in device memory
  int64_t nel;
  int Nx, Ny, Nz, bcmask;
  int rowchunks, tile_y;  // workgroup order: chunks per x-row (0: linear), y-tile height
  int nrhs;               // vectors applied at once (work item = element x vector)
  int64_t ld;             // distance between consecutive vectors, in values
  T h[3];
  const int* skip;        // continuous FE levels: the launch does nothing while *skip != 0 (NULL: never)
  double inv_nrhs;        // 1 / nrhs (the item -> element quotient, see item_elem)
  double inv_nx, inv_ny;  // 1 / Nx, 1 / Ny (element coordinates, see exact_div)
};

// The level's constant arguments (vectors unset, one vector, linear order).
template <typename T>
inline OpArgs<T> make_args(const hmg_level* L) {
  OpArgs<T> a;
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
  a.tabs = (const T*)L->tabs();
  a.nel = L->n_el;
  a.Nx = L->mesh.N[0];
  a.Ny = L->mesh.N[1];
  a.Nz = L->mesh.N[2];
  a.bcmask = L->mesh.bcmask();
  a.rowchunks = 0;
  a.tile_y = 1;
  a.nrhs = 1;
  a.inv_nrhs = 1.0;
  a.inv_nx = 1.0 / a.Nx;
  a.inv_ny = 1.0 / a.Ny;
  a.ld = L->n_dofs;
  for (int d = 0; d < 3; ++d) a.h[d] = (T)L->mesh.h(d);
  a.skip = nullptr;
  return a;
}

// Workgroup geometry of the operator kernels: 4 wavefronts whose lanes
// form groups of op_group_lanes(n) lanes (one wavefront, or for
// HMG_WIDE_GROUPS degrees the whole workgroup); a group owns
// lanes / n^2 elements (at least one), n^2 lanes each.  Whole-workgroup
// groups keep the lanes busy where n^2 leaves much of a wavefront over
// (n = 6: 36 of 64 lanes, 7 elements on 252 of 256), at the price of
// workgroup barriers between phases.
#ifndef HMG_WIDE_GROUPS
#define HMG_WIDE_GROUPS 0x40  // bit n: n = 6
#endif
constexpr int kOpWaves = 4;
constexpr int op_group_lanes(int n) { return ((HMG_WIDE_GROUPS >> n) & 1) ? 64 * kOpWaves : 64; }
constexpr int op_elems_per_group(int n) {
  return op_group_lanes(n) / (n * n) >= 1 ? op_group_lanes(n) / (n * n) : 1;
}
constexpr int op_elems_per_block(int n) { return 64 * kOpWaves / op_group_lanes(n) * op_elems_per_group(n); }
// LDS values of one n^3 array of an element (n = 8: rows of 9, planes of 72).
constexpr int lds_array_size(int n) { return n == 8 ? 8 * 72 : n * n * n; }
// Wavefront partial sums an OP_DOT launch on a mesh of nx x ny x nz
// elements can write: ceil(nx / EB) workgroups per x-row (EB >= 4), four
// wavefronts each, at most n_el + 4 ny nz.
inline int64_t op_partials_capacity(int nx, int ny, int nz) {
  const int64_t c = (int64_t)nx * ny * nz + (int64_t)kOpWaves * ny * nz + 64;
  return c > kPartials ? c : kPartials;
}

// One mesh of a multi-mesh launch (device table entry).  The work of a
// launch is a list of tiles; a tile is q consecutive workgroup chunks
// (op_elems_per_block(n) work items each) of one mesh.
template <typename T>
struct MeshEntry {
  OpArgs<T> a;     // the level's arguments; vector pointers unset
  int64_t off;     // first value of the mesh's block in the packed vectors
  int64_t tile0;   // first tile of the mesh in its launch
  int64_t chunks;  // workgroup chunks of the mesh
  int n;           // nodes per direction
  int id;          // mesh index in the batch (Chebyshev coefficient row)
};
// The host writes the table that the kernels read: the layout must agree in
// the host and the device compilation.
static_assert(sizeof(MeshEntry<double>) == 248 && sizeof(MeshEntry<float>) == 232, "MeshEntry layout");
static_assert(offsetof(MeshEntry<double>, off) == 216 && offsetof(MeshEntry<float>, off) == 200, "MeshEntry layout");
static_assert(offsetof(OpArgs<double>, ld) == 152 && offsetof(OpArgs<float>, h) == 152, "OpArgs layout");

// One multi-mesh launch: meshes table[0..count) (device memory, vector
// pointers resolved by multi_resolve), tiles split over the 8 XCDs at
// xcd[0..8] (device memory), `grid` workgroups (a multiple of 8).
struct MultiLaunch {
  const void* table;
  int count;
  int q;             // chunks per tile (1 unless persistent)
  const int64_t* xcd;
  unsigned grid;
  bool persist;      // workgroups loop over tiles (else one tile each)
};
// Set the vector pointers of table[0..count) for one launch: mesh i works on
// u + off_i, out + off_i, b + off_i, xold + off_i, and in Chebyshev mode
// takes sigma, theta = coef[id_i * cstride + 2 step + {0, 1}].
int multi_resolve(int prec, void* table, int count, const void* u, void* out, const void* b,
                  const void* xold, const void* coef, int cstride, int step, hipStream_t s);
// Launch over meshes that share n (nodes per direction), precision and
// geometry kind; modes OP_APPLY, OP_RESID, OP_CHEB.
int multi_launch(int n, int prec, bool curved, int mode, const MultiLaunch& m, hipStream_t s);
// Launch over Cartesian meshes of any degree in one kernel.
int fused_launch(int prec, int mode, const MultiLaunch& m, hipStream_t s);
// Resident workgroups per CU of those kernels (0 on error).
int multi_occupancy(int n, int prec, bool curved, int mode);
int fused_occupancy(int prec, int mode);

// DG: out = f(A u); FE: cell part into scratch, then node sum with the mode.
// OP_CHEB: out = u + sigma (u - xold) + theta dinv (b - A u)  (out may alias xold; xold NULL: x_old = 0)
// OP_DOT : out = A u, partials[blk] = sum u.(A u) (for p^T A p).
int launch_operator(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                    const void* xold, double sigma, double theta, int* nparts, hipStream_t s);
// The same for nrhs vectors at once: vector r of u, out, b, xold starts
// r*ld values after the first; dinv is shared.  Continuous FE levels with
// nrhs > 1 need fe_results, a block of nrhs * n_dg values of the level
// precision for the element-local results.  OP_DOT with nrhs > 1 (DG levels
// of degree 6 and 7: a group is one wavefront holding one element) writes
// one partial of u.(A u) per work item (element e, vector r) at e * nrhs + r
// of fe_results, a block of n_el * nrhs doubles (reduce_strided sums them).
int launch_operator_batched(const hmg_level* L, int mode, int nrhs, int64_t ld, const void* u, void* out,
                            const void* b, const void* xold, double sigma, double theta, int* nparts,
                            hipStream_t s, void* fe_results = nullptr);

// launch_operator (OP_APPLY) with the element-local results of a continuous
// FE level written to and summed from `scratch` (at least n_dg values of
// the level precision) instead of the level's own buffer; DG levels use
// no such buffer and ignore it.
int launch_operator_scratch(const hmg_level* L, const void* u, void* out, void* scratch, hipStream_t s);

// launch_operator with a device gate: on continuous FE levels every kernel
// of the apply returns at once while *skip != 0 (DG levels ignore it).
int launch_operator_gated(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                          const int* skip, hipStream_t s);
// Jacobi-preconditioned CG steps with FP64 scalars in device memory; every
// kernel returns at once while *skip != 0.
int ccg_init(int prec, const void* b, const void* dinv, void* x, void* r, void* z, void* p, int64_t n,
             const int* skip, hipStream_t s);
int ccg_xr(int prec, void* x, void* r, void* z, const void* p, const void* q, const void* dinv, int64_t n,
           const double* rz, const double* pq, const int* skip, hipStream_t s);
int ccg_p(int prec, void* p, const void* z, int64_t n, const double* rzn, const double* rz, const int* skip,
          hipStream_t s);
// *skip = 1 once *rzn <= tol2 * *rz0 (or not finite); *iters counts the iterations run
int ccg_check(const double* rzn, const double* rz0, double tol2, int* skip, int* iters, hipStream_t s);
// dot product that does nothing while *skip != 0
int vec_dot_gated(int prec, const void* x, const void* y, int64_t n, double* partials, double* out,
                  const int* skip, hipStream_t s);
// *skip = (gate[0] <= accept^2 gate[1] and finite); a rejected gate adds one to *fallbacks;
// *accepted (if not NULL) receives the same decision
int gate_to_skip(const double* gate, double accept, int* skip, int* fallbacks, hipStream_t s,
                 int* accepted = nullptr);
int set_flag(int* flag, int v, hipStream_t s);

// vectors (type by prec); n elements
int vec_fill(int prec, void* x, double a, int64_t n, hipStream_t s);
int vec_copy(int prec, const void* x, void* y, int64_t n, hipStream_t s);
int vec_axpby(int prec, double a, const void* x, double b, const void* y, void* z, int64_t n,
              hipStream_t s);  // z = a x + b y
int vec_recip(int prec, const void* x, void* y, int64_t n, hipStream_t s);       // y = 1/x
int vec_mul3(int prec, double a, const void* d, const void* b, void* z, int64_t n,
             hipStream_t s);  // z = a d .* b
int vec_convert(int from, const void* x, int to, void* y, int64_t n, hipStream_t s);
// the same, doing nothing while *skip != 0
int vec_convert_gated(int from, const void* x, int to, void* y, int64_t n, const int* skip, hipStream_t s);
// deterministic two-stage dot: result to dev double* out (and nparts returned)
int vec_dot(int prec, const void* x, const void* y, int64_t n, double* partials, double* out,
            hipStream_t s);
int reduce_partials(const double* partials, int nparts, double* out, hipStream_t s);
// out[r] = sum over j < n of partials[r + nrhs * j], r < nrhs (fixed order;
// tmp: nrhs * kPartialsB values)
int reduce_strided(const double* partials, int64_t n, int nrhs, double* out, double* tmp, hipStream_t s);
// CG updates with device scalars (all FP64): see kernels for formulas
// omega = *num / *den; x += omega p; r -= omega v; *save = *num if save;
// returns the number of partials of r.r written (>0) or an error (<0)
int cg_update_xr(double* x, double* r, const double* p, const double* v, const double* num,
                 const double* den, int64_t n, double* partials, hipStream_t s, double* save = nullptr,
                 float* r32 = nullptr);  // r32: r rounded to FP32 as well (may be NULL)
// *out = x . z with z in FP32, products in FP64 (as vec_dot)
int vec_dot_zf(const double* x, const float* z, int64_t n, double* partials, double* out, hipStream_t s);
// p = z + (*num / *den) p with z in FP32 (den NULL: p = z)
int cg_update_p_zf(double* p, const float* z, const double* num, const double* den, int64_t n, hipStream_t s);
// p = z + beta p, beta = *num / *den (negated if `negate`)
int cg_update_p(double* p, const double* z, const double* num, const double* den, int64_t n,
                hipStream_t s, bool negate = false);

// Several vectors (vector r starts r * ld values after the first), one
// launch each; per-vector FP64 scalars are arrays indexed by r and
// active[r] == 0 leaves vector r unchanged.
int vec_convert_b(int from, const void* x, int64_t ldx, int to, void* y, int64_t ldy, int64_t n, int nrhs,
                  hipStream_t s);
int vec_mul3_b(int prec, double a, const void* d, const void* b, void* z, int64_t n, int64_t ld, int nrhs,
               hipStream_t s);  // z_r = a d .* b_r
// out[r] = x_r . y_r (partials: nrhs * kPartialsB values)
int vec_dot_b(const double* x, const double* y, int64_t n, int64_t ld, int nrhs, double* partials, double* out,
              hipStream_t s);
// omega_r = num[r] / den[r]; x_r += omega_r p_r; r_r -= omega_r v_r; rr[r] = r_r . r_r; save[r] = num[r];
// r32 (may be NULL): every r_r rounded to FP32 as well, vector r at r * ld32;
// x = NULL: the x step is deferred, omega_r stored in alpha[r] (cg_update_p_zf_b
// or cg_step_x_b take it)
int cg_update_xr_b(double* x, double* r, const double* p, const double* v, const double* num, const double* den,
                   int64_t n, int64_t ld, int nrhs, double* partials, double* rr, double* save, const int* active,
                   hipStream_t s, float* r32 = nullptr, int64_t ld32 = 0, double* alpha = nullptr);
// out[r] = x_r . z_r with z in FP32 (vector r at r * ldz), products in FP64
int vec_dot_zf_b(const double* x, const float* z, int64_t n, int64_t ld, int64_t ldz, int nrhs, double* partials,
                 double* out, hipStream_t s);
// p_r = z_r + (num[r] / den[r]) p_r with z in FP32 (den NULL: p_r = z_r);
// x != NULL: first x_r += alpha[r] p_r (the deferred step of the last update)
int cg_update_p_zf_b(double* p, const float* z, const double* num, const double* den, int64_t n, int64_t ld,
                     int64_t ldz, int nrhs, const int* active, hipStream_t s, double* x = nullptr,
                     const double* alpha = nullptr);
// x_r += alpha[r] p_r for the vectors r set in mask (deferred steps)
int cg_step_x_b(double* x, const double* p, const double* alpha, int64_t n, int64_t ld, int nrhs, uint64_t mask,
                hipStream_t s);
// p_r = z_r + beta_r p_r, beta_r = num[r] / den[r] (negated if `negate`)
int cg_update_p_b(double* p, const double* z, const double* num, const double* den, int64_t n, int64_t ld, int nrhs,
                  const int* active, bool negate, hipStream_t s);

// transfers (element-local tensor-product kernels); nrhs vectors in one
// launch, vector r of each block r * ld_* values after the first
// DG p / h: fine += P coarse, coarse = P^T fine
int tr_dg_prolongate(int prec, int kind, int nf, int nc, const int Nf[3], const double* P0,
                     const double* P1, const void* coarse, void* fine, int add, hipStream_t s, int nrhs = 1,
                     int64_t ld_c = 0, int64_t ld_f = 0);
int tr_dg_restrict(int prec, int kind, int nf, int nc, const int Nf[3], const double* P0,
                   const double* P1, const void* fine, void* coarse, hipStream_t s, int nrhs = 1,
                   int64_t ld_f = 0, int64_t ld_c = 0);
// c-transfers between the FE vector and a DG-layout vector on the same mesh
//   inject: dg = E(free * w * fe) with w = 1 or 1/mult;  add: dg += ... if add
//   sum   : fe (+)= free * w * E^T dg
int tr_c_inject(int prec, const Mesh& m, int k, const void* fe, void* dg, int weight_mult,
                int add, hipStream_t s, int nrhs = 1, int64_t ld_fe = 0, int64_t ld_dg = 0);
int tr_c_sum(int prec, const Mesh& m, int k, const void* dg, void* fe, int weight_mult, int add,
             hipStream_t s, int nrhs = 1, int64_t ld_dg = 0, int64_t ld_fe = 0);
// FE operator node sum with a mode (see launch_operator) for nrhs vectors
// in one launch: vector r of u, out, b, xold starts r * ld values after the
// first, its element-local results r * n_dg values after the first
// (scratch: the element-local results, NULL for the level's own buffer)
int fe_node_sum(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                const void* xold, double sigma, double theta, hipStream_t s, const int* skip = nullptr,
                const void* scratch = nullptr, int nrhs = 1, int64_t ld = 0);
// coarse dense FP64 inverse apply: x = Ainv b (b, x of prec), n unknowns
int coarse_gemv(int prec, const double* Ainv, const void* b, void* x, int n, hipStream_t s);
// SplitMix64 uniform [-1,1) vector
int vec_splitmix(int prec, uint64_t seed, void* x, int64_t n, hipStream_t s);

}  // namespace hmg
