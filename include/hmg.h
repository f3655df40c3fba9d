/*
 * hmg.h — C ABI of the MI355X (gfx950) matrix-free SIPG operator and hybrid
 * multigrid solver for the 3-D Poisson equation.
 *
 * Method: Fehn, Munch, Wall, Kronbichler, "Hybrid multigrid methods for
 * high-order discontinuous Galerkin discretizations", arXiv:1910.01900.
 * Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 *  - All vectors and all device memory belong to the caller.  The library
 *    never allocates device memory: persistent device state of a handle
 *    (geometry, penalty, inverse diagonal, level vectors, coarse inverse)
 *    lives in a workspace the caller binds after asking for its size.
 *    Workspaces must stay alive and untouched until the handle is destroyed.
 *  - Vector arguments are device pointers, 256-byte aligned, contiguous,
 *    of the handle's precision (double for HMG_F64, float for HMG_F32)
 *    unless stated otherwise.
 *  - Work is enqueued on the given HIP stream (0 = legacy default stream)
 *    and is stream-ordered; calls return before the GPU finishes unless the
 *    entry point says "blocks".
 *  - Every call returns an hmg_status.  Negative values are errors and leave
 *    outputs unspecified; hmg_last_error() returns a thread-local message.
 *  - Handles are not thread-safe for concurrent mutation.  Two calls that
 *    use the same handle's workspace on different streams race.
 *
 * Layouts
 *  - Elements of an Nx x Ny x Nz box: e = ex + Nx*(ey + Ny*ez).
 *  - DG vector (discontinuous Q_k, n = k+1): index e*n^3 + i + n*(j + n*l),
 *    (i, j, l) the GLL node indices in the reference directions x, y, z.
 *  - FE vector (continuous Q_k): global node index gx + Mx*(gy + My*gz),
 *    M_d = N_d*k + 1, gx = ex*k + i (etc.).  Nodes on Dirichlet box faces
 *    are present; the operator acts as the identity on them (Sec. 2).
 */
#ifndef HMG_H
#define HMG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HMG_OK = 0,
  HMG_NOT_CONVERGED = 1,      /* warning: results valid, tolerance not reached */
  HMG_ERR_INVALID = -1,       /* bad argument (null, size, range, alignment)   */
  HMG_ERR_UNSUPPORTED = -2,   /* valid but not implemented (degree, space, size) */
  HMG_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed    */
  HMG_ERR_BREAKDOWN = -4,     /* CG breakdown: p^T A p <= 0 (operator not SPD)  */
  HMG_ERR_NONFINITE = -5,     /* NaN or Inf met in a residual norm             */
  HMG_ERR_WORKSPACE = -6      /* workspace missing, too small or misaligned    */
} hmg_status;

typedef enum { HMG_F64 = 0, HMG_F32 = 1 } hmg_prec;
typedef enum { HMG_DG = 0, HMG_FE = 1 } hmg_space;

/* Thread-local text of the last error (empty string if none). */
const char* hmg_last_error(void);

/* Library version: major*10000 + minor*100 + patch.  0.1.0 (100): levels,
 * transfers, hierarchy, PCG; 0.2.0 (200): several vectors per launch,
 * recorded graphs, multi-mesh batches, the learned coarse correction;
 * 0.3.0 (300): the iterative coarse solve (HMG_COARSE_CG,
 * hmg_hierarchy_set_coarse_cg) for coarse levels without a dense inverse;
 * 0.4.0 (400): several right-hand sides per solve (hmg_pcg_solve_batched,
 * hmg_vcycle_batched), the operator apply without allocation
 * (hmg_operator_apply_noalloc), the FP64 iterative coarse solve. */
int hmg_version(void);

/*
 * Structured hexahedral mesh of the box [lo, hi] (Sec. 2 and Sec. 5.3).
 *  nel[3]       elements per direction, each >= 1.
 *  degree       polynomial degree k of the shape functions, 1..7.
 *  deformed     0: Cartesian (affine) mesh; 1: curvilinear mesh whose points
 *               are moved by x_i += deform_amp * prod_j sin(deform_waves*pi*s_j),
 *               s_j = (x_j - lo_j)/(hi_j - lo_j), represented by a degree-3
 *               (Q3) mapping interpolating the deformation at the 4^3 GLL
 *               support points of each element (Sec. 5.3: cubic mapping),
 *               or exactly (mapping_degree 0).
 *  bc[6]        per box face (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi):
 *               0 Dirichlet (weak, mirror principle, Sec. 2), 1 Neumann.
 *  ip_factor    multiplies the penalty tau_e (Sec. 2; Table 8 varies it).
 *  tau_scale    optional host array of N_el per-element penalty factors
 *               (copied during create; may be NULL).
 *  mapping_degree  3: the degree-3 mapping above (Sec. 5.3); 0: the
 *               analytic deformation itself (exact geometry).  Other values:
 *               HMG_ERR_UNSUPPORTED.  (Added in 0.4.0: callers must set it.)
 */
typedef struct {
  int32_t nel[3];
  double lo[3], hi[3];
  int32_t degree;
  int32_t deformed;
  double deform_amp;
  int32_t deform_waves;
  uint8_t bc[6];
  double ip_factor;
  const double* tau_scale;
  int32_t mapping_degree;
} hmg_mesh_desc;

typedef struct hmg_level hmg_level;
typedef struct hmg_transfer hmg_transfer;
typedef struct hmg_hierarchy hmg_hierarchy;

/*
 * One multigrid level: a discretization (space, degree, mesh, precision) of
 * the homogeneous Laplace operator (Sec. 2: re-discretization on each level).
 * create builds geometry and penalty on the host; query reports the DoF
 * count and the workspace size; bind uploads to the workspace and computes
 * the inverse diagonal (blocks until done).
 */
int hmg_level_create(const hmg_mesh_desc* mesh, int space, int prec, hmg_level** out);
int hmg_level_query(const hmg_level* L, int64_t* n_dofs, size_t* workspace_bytes);
int hmg_level_bind(hmg_level* L, void* dev_workspace, size_t bytes, hipStream_t stream);
void hmg_level_destroy(hmg_level* L);

/*
 * v = A u, the matrix-free operator of eq:MatrixFreeAbstractNotation (Sec. 4):
 * cell integrals by sum factorization plus, for DG, the interior-penalty
 * face integrals (jump, average, penalty; mirror boundary conditions).
 * u and v must not overlap.  v is overwritten.
 */
int hmg_operator_apply(const hmg_level* L, const void* u, void* v, hipStream_t stream);

/*
 * For callers that cannot allocate device memory at call time (work recorded
 * into HIP graphs, tight serving loops, harnesses that forbid allocation):
 * the operator of hmg_operator_apply, v = A u, with nothing allocated and no
 * workspace beyond the level's bound one.  On a continuous FE level the
 * element-local results (n_el (k+1)^3 values of the level precision) go to
 * a static device array of HMG_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends; levels needing more
 * return HMG_ERR_UNSUPPORTED before any launch.  DG levels need no such
 * buffer (the call equals hmg_operator_apply).  Results are bitwise equal
 * to hmg_operator_apply.  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must
 * be ordered by the caller.  Nothing in the array needs clearing: every
 * call writes all the values it reads.
 */
#define HMG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hmg_operator_apply_noalloc(const hmg_level* L, const void* u, void* v, hipStream_t stream);

/* r = b - A u (the residual of Alg. 2).  r must not overlap u. */
int hmg_residual(const hmg_level* L, const void* b, const void* u, void* r, hipStream_t stream);

/*
 * The operator of hmg_operator_apply on nrhs vectors in one launch (DG
 * levels only): v_r = A u_r for r = 0..nrhs-1, where vector r of each
 * argument starts r*ld values (of the level precision) after its first.
 * The element geometry is read once for all vectors of an element.
 * 1 <= nrhs <= 64; ld >= the level's DoF count, ld * value size a multiple
 * of 256 bytes.  Results equal nrhs separate hmg_operator_apply calls.
 * The u and v ranges must not overlap.  HMG_ERR_UNSUPPORTED on FE levels
 * and when the level's element count times nrhs reaches 2^31.
 */
int hmg_operator_apply_batched(const hmg_level* L, int nrhs, const void* u, void* v, int64_t ld,
                               hipStream_t stream);

/* r_r = b_r - A u_r for nrhs vectors (layout and limits as above). */
int hmg_residual_batched(const hmg_level* L, int nrhs, const void* b, const void* u, void* r,
                         int64_t ld, hipStream_t stream);

/* d = diag(A) (Sec. 3.1: the diagonal used by the Chebyshev-Jacobi smoother).
 * The diagonal is setup data: the library evaluates a(phi_i, phi_i) on the
 * host while creating the level (sum-factorized cell part plus own-side face
 * terms) and keeps it on the device after bind; this call copies it. */
int hmg_diagonal(const hmg_level* L, void* d, hipStream_t stream);
/* Host copy of diag(A) (out: host array of n_dofs doubles); usable before bind. */
int hmg_level_diagonal_host(const hmg_level* L, double* out);

/*
 * Estimate lambda_max of D^{-1}A by `iters` Jacobi-preconditioned CG
 * iterations (Sec. 3.1: 20 iterations) from the start vector drawn by the
 * SplitMix64 generator seeded with `seed` (value i = 2*top53bits*2^-53 - 1
 * of output i+1); returns the largest Ritz value.  Blocks.
 */
int hmg_estimate_lambda_max(const hmg_level* L, int iters, uint64_t seed, double* lmax,
                            hipStream_t stream);

/*
 * Alg. 3: `degree` steps of Chebyshev-accelerated Jacobi on A x = b with
 * eigenvalue interval [lo_frac, hi_frac] * lmax (Sec. 3.1: 0.06 and 1.2);
 * sigma_j, theta_j of the classical three-term Chebyshev iteration.
 * x holds x_0 on entry (ignored if x_is_zero) and x_degree on exit.
 * Uses one level-internal temporary vector.
 */
int hmg_chebyshev_smooth(const hmg_level* L, const void* b, void* x, int degree, double lmax,
                         double lo_frac, double hi_frac, int x_is_zero, hipStream_t stream);

/*
 * Transfer between two levels that differ in exactly one of (h, p, c)
 * (Sec. 3.2).  kind 'p': same mesh and space, coarse degree < fine degree;
 * 'h': same degree and space, coarse mesh = fine mesh with every N_d
 * halved; 'c': fine DG and coarse FE on the same mesh and degree.
 * Both levels must have the same precision and be bound; the transfer needs
 * a workspace for its DG-layout temporaries (FE transfers only).
 */
int hmg_transfer_create(const hmg_level* fine, const hmg_level* coarse, char kind, hmg_transfer** out);
int hmg_transfer_query(const hmg_transfer* T, size_t* workspace_bytes);
int hmg_transfer_bind(hmg_transfer* T, void* dev_workspace, size_t bytes);
void hmg_transfer_destroy(hmg_transfer* T);
/* fine += P coarse, P = sum_e S_e P_e G_e (multiplicity-weighted scatter). */
int hmg_prolongate_add(const hmg_transfer* T, const void* coarse, void* fine, hipStream_t stream);
/* coarse = P^T fine (overwrite). */
int hmg_restrict(const hmg_transfer* T, const void* fine, void* coarse, hipStream_t stream);

/*
 * Hybrid multigrid hierarchy (Sec. 3.2) for the DG discretization of `mesh`.
 *  strategy      letters in coarsening order, e.g. "p", "cph", "hpc" (Table 4);
 *                each letter coarsens exhaustively in its turn.
 *  pseq          p-sequence: 0 p-1, 1 floor(p/2), 2 straight to 1 (Sec. 3.2.2).
 *  h_min         h-coarsening stops when an N_d is odd or max N_d <= h_min.
 *  smoother_degree  Chebyshev steps per smoothing (Sec. 3.1: 5).
 *  mg_prec       precision of the V-cycle (smoothers, transfers, level
 *                operators); the coarsest-level solve is always FP64.  The
 *                outer PCG always runs in FP64 with its own FP64 fine operator.
 *  lmax_seed     seed of the lambda_max start vectors (level l uses seed + l).
 * The coarse solver is an exact FP64 solve: the coarsest operator is probed
 * column by column on the GPU, factored (Cholesky) on the host and its
 * inverse applied as a dense matrix-vector product (at most 8192 unknowns).
 * bind uploads everything, estimates lambda_max per level and factors the
 * coarse matrix; it blocks.
 */
int hmg_hierarchy_create(const hmg_mesh_desc* mesh, const char* strategy, int pseq, int h_min,
                         int smoother_degree, int mg_prec, uint64_t lmax_seed,
                         hmg_hierarchy** out);
int hmg_hierarchy_query(const hmg_hierarchy* H, int64_t* n_dofs, size_t* workspace_bytes);
int hmg_hierarchy_bind(hmg_hierarchy* H, void* dev_workspace, size_t bytes, hipStream_t stream);
void hmg_hierarchy_destroy(hmg_hierarchy* H);

/* Level l (0 = finest) of the V-cycle: space, degree, mesh size, DoFs and
 * the lambda_max estimate used by its smoother (coarsest level: lmax 0). */
typedef struct {
  int32_t space, degree, nel[3], prec;
  int64_t n_dofs;
  double lmax;
} hmg_level_info;
int hmg_hierarchy_levels(const hmg_hierarchy* H, int* n_levels);
int hmg_hierarchy_level_info(const hmg_hierarchy* H, int l, hmg_level_info* info);
/* Override the lambda_max of level l (e.g. to replay another estimate). */
int hmg_hierarchy_set_lmax(hmg_hierarchy* H, int l, double lmax);

/*
 * x = M^{-1} b: one V-cycle of Alg. 2 with x^(L) = 0 (Sec. 3: the PCG
 * preconditioner).  b and x are FP64 vectors on the finest level (converted
 * to and from mg_prec internally).  b and x must not overlap.
 */
int hmg_vcycle(hmg_hierarchy* H, const double* b, double* x, hipStream_t stream);

/*
 * For callers whose meshes are small enough that kernel launch latency
 * dominates (Sec. 5 strong-scaling regime): with enable != 0, hmg_pcg_solve
 * records one iteration after the first (V-cycle of Alg. 2, the dot
 * products and vector updates of Alg. 1, the operator apply) and hmg_vcycle
 * records its V-cycle, each once as a HIP graph on a stream the library
 * creates (default priority), and replays it on the caller's stream.  A
 * recording is redone when the solution (and, for hmg_vcycle, right-hand
 * side) pointers change or the hierarchy is bound again.  Results are
 * bitwise identical to enable = 0.  Calls on one hierarchy must not overlap.
 */
int hmg_hierarchy_set_graph(hmg_hierarchy* H, int enable);

typedef struct {
  int32_t iters;
  double r0, rn;       /* ||b - A x_0||_2 and final ||r||_2 */
  double rho, n10;     /* Sec. 5.1: (rn/r0)^(1/iters), -10/log10(rho) */
} hmg_solve_stats;

/*
 * Alg. 1: preconditioned CG in FP64 with one V-cycle as preconditioner.
 * Stops when ||r||/||r_0|| <= rtol or ||r|| <= atol.  x holds x_0 on entry
 * and the solution on exit.  Blocks (one device-to-host read of ||r|| per
 * iteration).  Returns HMG_NOT_CONVERGED after maxit iterations,
 * HMG_ERR_BREAKDOWN if p^T A p <= 0 and HMG_ERR_NONFINITE on NaN/Inf;
 * stats (may be NULL) are filled in every case.
 */
int hmg_pcg_solve(hmg_hierarchy* H, const double* b, double* x, double rtol, double atol,
                  int maxit, hmg_solve_stats* stats, hipStream_t stream);

/*
 * Several right-hand sides solved together (Alg. 1 and Alg. 2 for each
 * vector, with its own scalars): the vectors travel through every level of
 * the V-cycle as one block: every operator application of the smoothers,
 * the residuals and the outer CG takes all vectors in one launch, reading
 * the element geometry once for all of them (on continuous FE levels the
 * node sums of all vectors follow as one launch), and so does each grid
 * transfer kernel; the coarse solve takes the vectors one after another.
 * A level whose element count
 * times nrhs reaches 2^31 returns HMG_ERR_UNSUPPORTED.
 * set_max_rhs (1..64, default 1) reserves workspace for up to max_rhs
 * vectors and must precede hmg_hierarchy_query and _bind.
 * Vector q of b and x starts q*ld values after the first (FP64, device;
 * ld >= n_dofs, ld*8 a multiple of 256; b and x must not overlap).
 * hmg_pcg_solve_batched: x holds the start vectors on entry; each vector
 * stops, and is left unchanged from then on, when its own ||r||/||r_0|| <=
 * rtol or ||r|| <= atol; the call returns when all have stopped or after
 * maxit iterations (HMG_NOT_CONVERGED if any has not).  After
 * HMG_ERR_NONFINITE the contents of x are unspecified.  stats (nrhs
 * entries, may be NULL) as for hmg_pcg_solve.  Blocks.  The learned coarse
 * solve is not available here (HMG_ERR_UNSUPPORTED).  nrhs must not
 * exceed max_rhs; with max_rhs = 1 (nothing reserved; nrhs up to 64) or
 * nrhs = 1 the call runs hmg_pcg_solve (hmg_vcycle) for each vector.
 */
int hmg_hierarchy_set_max_rhs(hmg_hierarchy* H, int max_rhs);
int hmg_vcycle_batched(hmg_hierarchy* H, int nrhs, const double* b, double* x, int64_t ld, hipStream_t stream);
int hmg_pcg_solve_batched(hmg_hierarchy* H, int nrhs, const double* b, double* x, int64_t ld, double rtol,
                          double atol, int maxit, hmg_solve_stats* stats, hipStream_t stream);

/*
 * Manufactured right-hand side for u = prod_j sin(freq * x_j):
 * f = 3 freq^2 u and Dirichlet data g = u moved to the right-hand side as in
 * Sec. 2 (b_i = (phi_i, f) - sum_{Dirichlet F} (dphi_i/dn - 2 tau phi_i, g)_F).
 * Computed on the host during the call and copied to b (DG levels only;
 * b has the level's precision).  Blocks.
 */
int hmg_rhs_sine(const hmg_level* L, double freq, void* b, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned coarse-grid correction.  A U-Net (3x3x3 convolutions on a G^3
 * grid, G a multiple of 8; levels G, G/2, G/4, G/8 with 16, 32, 48, 48
 * channels; 2x2x2 average pooling, nearest upsampling with skip addition;
 * ReLU except the last layer; about 181k parameters) maps the coarse
 * residual of a continuous Q1 coarsest level (its nodes placed at the grid
 * points, input channels: residual / its RMS, free-node mask) to the
 * correction (times RMS times the scale of hmg_hierarchy_coarse_info).
 * Convolutions run on the BF16 matrix cores with FP32 accumulation; the
 * parameters, Adam state and activations are FP32.  Parameters are packed
 * per layer as w[cout][27][cin] (tap t = (dx+1) + 3 (dy+1) + 9 (dz+1))
 * followed by b[cout].  Training pairs come from the method's own exact
 * FP64 coarse solves (hmg_hierarchy_capture, _coarse_solve_batch,
 * _learned_data).  Inputs in[batch][G^3][2], outputs / targets
 * [batch][G^3] (FP32, device, 256-byte aligned).
 */
typedef struct hmg_net hmg_net;
/* grid 8..64 (multiple of 8), max_batch 1..4096; weights He-uniform from
 * SplitMix64(seed) at bind, biases 0. */
int hmg_net_create(int grid, int max_batch, uint64_t seed, hmg_net** out);
int hmg_net_query(const hmg_net* N, int64_t* n_params, size_t* workspace_bytes);
int hmg_net_bind(hmg_net* N, void* dev_workspace, size_t bytes, hipStream_t stream);
void hmg_net_destroy(hmg_net* N);
/* Copy the n_params FP32 parameters out of / into the network (device). */
int hmg_net_get_params(const hmg_net* N, float* dst, hipStream_t stream);
int hmg_net_set_params(hmg_net* N, const float* src, hipStream_t stream);
int hmg_net_forward(hmg_net* N, const float* in, float* out, int batch, hipStream_t stream);
/* Loss (mean over the masked points of (out - target)^2, FP64 device
 * scalar) and its gradient with respect to every parameter (device, FP32,
 * packed like the parameters); nothing is updated. */
int hmg_net_gradient(hmg_net* N, const float* in, const float* target, int batch, float* grad,
                     double* loss, hipStream_t stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) at learning rate lr; *loss
 * (device, may be NULL) receives the loss before the step. */
int hmg_net_train_step(hmg_net* N, const float* in, const float* target, int batch, double lr,
                       double* loss, hipStream_t stream);

enum { HMG_COARSE_EXACT = 0, HMG_COARSE_SMOOTH = 1, HMG_COARSE_LEARNED = 2, HMG_COARSE_CG = 3 };
/*
 * Coarsest-level solve of the V-cycle: EXACT (dense FP64 inverse; coarse
 * levels up to 8192 unknowns, the default there), CG (Jacobi-preconditioned
 * CG in FP64 on an FP64 copy of the coarsest level, whatever the V-cycle
 * precision, to hmg_hierarchy_set_coarse_cg's tolerance; the default above
 * 8192 unknowns), SMOOTH (Chebyshev smoothing only, the
 * V-cycle without a coarse solve) or LEARNED: x = network(b), checked on the
 * GPU by |b - A x| <= accept |b| (finite), else the exact solve or, without
 * a dense inverse, the CG solve (fallbacks counted, hmg_hierarchy_coarse_stats).
 * LEARNED needs a continuous Q1 coarsest level whose node grid fits the
 * network's grid.  LEARNED and CG switch hmg_pcg_solve to flexible CG (the
 * preconditioner changes between iterations).
 * HMG_ERR_UNSUPPORTED: EXACT without a dense inverse.
 */
int hmg_hierarchy_set_coarse(hmg_hierarchy* H, int mode, hmg_net* net, double accept);
/* Iterative coarse solve: stop at |r.z| <= rtol^2 |r_0.z_0| or after maxit
 * iterations (defaults 1e-3, 50); converged iterations cost empty launches. */
int hmg_hierarchy_set_coarse_cg(hmg_hierarchy* H, double rtol, int maxit);
/* Flexible CG (beta = -(z_{k+1} . A p_k) / (p_k . A p_k)); equal to PCG in
 * exact arithmetic for a fixed symmetric preconditioner. */
int hmg_hierarchy_set_flexible(hmg_hierarchy* H, int enable);
/* Coarse unknowns n, node grid (0 for a DG coarsest level) and the output
 * scale of the learned correction (1 / mean free diagonal). */
int hmg_hierarchy_coarse_info(const hmg_hierarchy* H, int64_t* n, int* Mx, int* My, int* Mz, double* scale);
/* Copy the coarsest right-hand side of every following V-cycle (FP64, n
 * values each, at most capacity) to buf; capacity 0 stops.  V-cycles of
 * several right-hand sides (hmg_vcycle_batched, hmg_pcg_solve_batched)
 * contribute one per vector.  V-cycles run without recorded graphs while
 * capturing. */
int hmg_hierarchy_capture(hmg_hierarchy* H, double* buf, int capacity);
int hmg_hierarchy_captured(const hmg_hierarchy* H, int* count);
/* E[s] = A_c^{-1} R[s] for count coarse vectors (FP64, n values each): the
 * dense inverse, or FP64 Jacobi-PCG to 1e-12 without one (blocks). */
int hmg_hierarchy_coarse_solve_batch(const hmg_hierarchy* H, const double* R, double* E, int count,
                                     hipStream_t stream);
/* Network inputs (and targets if target != NULL) of count <= 1024 coarse
 * vectors R (and exact corrections E) for a grid of `grid` points. */
int hmg_hierarchy_learned_data(const hmg_hierarchy* H, int grid, const double* R, const double* E, int count,
                               float* in, float* target, hipStream_t stream);
/* Number of learned coarse solves replaced by the exact one since bind. Blocks. */
int hmg_hierarchy_coarse_stats(const hmg_hierarchy* H, int* fallbacks, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batches: many independent DG meshes of uneven size and degree, nrhs
 * vectors each, under one schedule of launches.  The operator of every mesh
 * is the one of hmg_operator_apply (Sec. 4, eq:MatrixFreeAbstractNotation);
 * the Chebyshev smoother is Alg. 3 on every mesh with its own lambda_max.
 *
 * Packed multi-vectors: one device buffer of total_values values (level
 * precision, 256-byte aligned) holds, for mesh i, vector r (0 <= r < nrhs)
 * at offset_i + r * ld_i (hmg_batch_layout; ld_i is the mesh's DoF count
 * rounded up to 256 bytes, values between n_dofs and ld_i are not read
 * and are left unchanged).
 *
 * The levels stay owned by the caller; they must share the precision, be DG
 * levels, outlive the batch and be bound before the batch is bound (bind
 * the batch again after re-binding a level).  Calls on one batch must not
 * overlap.
 */
typedef struct hmg_batch hmg_batch;

/* HMG_ERR_INVALID: NULL levels, count < 1, nrhs outside 1..64, mixed
 * precision; HMG_ERR_UNSUPPORTED: an FE level or a mesh too large. */
int hmg_batch_create(const hmg_level* const* levels, int count, int nrhs, hmg_batch** out);
int hmg_batch_query(const hmg_batch* B, int64_t* total_values, size_t* workspace_bytes);
int hmg_batch_layout(const hmg_batch* B, int i, int64_t* offset, int64_t* ld);
/* Uploads the mesh tables into ws (device, 256-byte aligned, at least
 * workspace_bytes) and selects the default schedule (one launch per
 * degree group, one workgroup per tile).  Blocks. */
int hmg_batch_bind(hmg_batch* B, void* dev_workspace, size_t bytes, hipStream_t stream);
void hmg_batch_destroy(hmg_batch* B);

/*
 * Schedule.  single = 1: one launch over all meshes (Cartesian meshes only,
 * else HMG_ERR_UNSUPPORTED); single = 0: one launch per (degree, geometry)
 * group.  persistent = 1: at most blocks_per_cu workgroups per CU loop over
 * tiles of chunks_per_tile (1, 2 or 4) workgroup chunks; persistent = 0:
 * one workgroup per tile, chunks_per_tile must be 1.  Results do not depend
 * on the schedule.
 */
int hmg_batch_set_schedule(hmg_batch* B, int single, int persistent, int chunks_per_tile,
                           int blocks_per_cu);
/* Times every candidate schedule of each launch with `reps` applies of u
 * into v (packed vectors, v is overwritten) on `stream` and keeps the
 * fastest; *best_ms (may be NULL) receives the time of one batch apply.
 * Blocks. */
int hmg_batch_autotune(hmg_batch* B, const void* u, void* v, int reps, hipStream_t stream,
                       double* best_ms);
int hmg_batch_schedule(const hmg_batch* B, int* single, int* units);
/* Launch u of the schedule: nodes per direction n (0 for the single
 * launch), geometry kind, mesh count, persistent, chunks per tile,
 * workgroups per CU, grid size and its autotuned time (-1 if not tuned). */
int hmg_batch_unit_info(const hmg_batch* B, int u, int* n, int* curved, int* meshes, int* persistent,
                        int* chunks_per_tile, int* blocks_per_cu, unsigned* grid, double* ms);

/* v = A u for every mesh and vector (packed vectors; u and v must not
 * overlap). */
int hmg_batch_apply(const hmg_batch* B, const void* u, void* v, hipStream_t stream);
/* r = b - A u (u and r must not overlap). */
int hmg_batch_residual(const hmg_batch* B, const void* b, const void* u, void* r, hipStream_t stream);
/* Chebyshev coefficients (Alg. 3, classical three-term recurrence on
 * [lo_frac, hi_frac] * lmax[i]) for every mesh i: lmax has count values.
 * Blocks. */
int hmg_batch_set_chebyshev(hmg_batch* B, const double* lmax, int degree, double lo_frac, double hi_frac,
                            hipStream_t stream);
/* degree Chebyshev steps on every mesh and vector, each one operator
 * launch fused with the update; x holds the start vector on entry and the
 * result on exit; tmp is a second packed vector; b, x, tmp must not
 * overlap. */
int hmg_batch_chebyshev_smooth(const hmg_batch* B, const void* b, void* x, void* tmp, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HMG_H */
