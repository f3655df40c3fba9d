// Operator kernels for gfx950 and their launchers: the single-mesh kernel
// (one launch per apply, several vectors per launch on DG levels) and the
// multi-mesh kernel (many meshes of one degree in one persistent launch).
// The per-wavefront operator body is in op_body.h.
#include "op_body.h"

namespace hmg {

#ifndef HMG_DISPATCH_ONLY
// ------------------------------------------------------------------ single mesh
template <int N, typename T, bool CURVED, bool FE, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(op_wpe<N, T, CURVED, FE>())))
op_kernel(const OpArgs<T> a) {
  using C = Cfg<N, CURVED, FE>;
  if constexpr (FE) {
    if (a.skip && *a.skip) return;  // gated apply (iterative coarse solve)
  }
  constexpr int WL = op_group_lds<N, T, CURVED, FE, MODE>();
  __shared__ T smem[C::GROUPS * WL];
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / C::GL);  // group-uniform (scalar)
  T* const W0 = smem + grp * WL;  // this group's LDS
  int count;
  const int64_t first = block_chunk(a, xcd_block(), C::EB, &count);
  const int64_t it0 = first + (int64_t)grp * C::EW;  // first item of the group
  load_lane_tables<T, C::LT, C::GL>(a.tabs, W0 + C::EW * C::PER);
  const double acc = op_items<N, T, CURVED, FE, MODE>(a, it0, count - grp * C::EW, W0);
  if constexpr (!FE && MODE == OP_DOT)
    if ((threadIdx.x & 63) == 0) {
      if (a.nrhs == 1)  // one partial per wavefront
        a.partials[(int64_t)blockIdx.x * C::WAVES + (threadIdx.x >> 6)] = acc;
      else if (it0 < a.nel * a.nrhs)  // one element per group: one partial per work item
        a.partials[it0] = acc;
    }
}

// ------------------------------------------------------------------ multi mesh
// Work of a multi-mesh launch: tiles of q workgroup chunks of one mesh.
// Workgroups are dispatched round-robin over the 8 XCDs; XCD x takes the
// contiguous tile range [xcd[x], xcd[x+1]) (ranges balanced by estimated
// cost on the host) and its workgroups stride through it, so the tiles of
// one mesh run on one L2 at the same time.  A workgroup loops until its
// range is exhausted (persistent when the grid is smaller than the tile
// count).
// Meshes of one degree and geometry kind (DG; apply, residual, Chebyshev).
// PERSIST: each workgroup loops over the tiles of its XCD's range with the
// grid's stride; otherwise the grid has a workgroup per tile of one chunk
// (q = 1) and the body is straight-line code, like the single-mesh kernel
// (the loop costs registers: loop state and hoisted lane arithmetic).
template <int N, typename T, bool CURVED, int MODE, bool PERSIST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Cfg<N, CURVED, false>::WPE)))
op_multi_kernel(const MultiArgs<T> m) {
  using C = Cfg<N, CURVED, false>;
  constexpr int WL = op_group_lds<N, T, CURVED, false, MODE>();
  __shared__ T smem[C::GROUPS * WL];
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / C::GL);  // group-uniform (scalar)
  T* const W0 = smem + grp * WL;
  const cptr<MeshEntry<T>> tab = (cptr<MeshEntry<T>>)(uintptr_t)m.table;
  const cptr<int64_t> xcd = (cptr<int64_t>)(uintptr_t)m.xcd;
  const int x = blockIdx.x & 7;
  const int64_t end = xcd[x + 1];
  int64_t tile = xcd[x] + (blockIdx.x >> 3);
  if (tile >= end) return;
  // every mesh of the launch has the same degree and precision: one table
  load_lane_tables<T, C::LT, C::GL>(tab[0].a.tabs, W0 + C::EW * C::PER);
  int mi = find_mesh(tab, m.count, tile);
  if constexpr (PERSIST) {
    const int64_t stride = gridDim.x >> 3;
    for (; tile < end; tile += stride) {
      while (mi + 1 < m.count && tab[mi + 1].tile0 <= tile) ++mi;
      multi_tile<N, T, CURVED, MODE>(m, tab + mi, tile, W0);
    }
  } else {
    const cptr<MeshEntry<T>> E = tab + mi;
    const OpArgs<T>& a = *(const OpArgs<T>*)&E->a;
    const int64_t it0 = (tile - E->tile0) * C::EB + (int64_t)grp * C::EW;
    op_items<N, T, CURVED, false, MODE>(a, it0, group_count(a, it0), W0);
  }
}

// ------------------------------------------------------------------ launchers
// y-tile height of the workgroup order (rows of elements)
static constexpr int kTileY = 4;

template <int N, typename T, bool CURVED, bool FE>
static int run_op(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                  const void* xold, double sigma, double theta, int* nparts, int nrhs, int64_t ld,
                  const int* skip, void* scratch, hipStream_t s) {
  using C = Cfg<N, CURVED, FE>;
  OpArgs<T> a = make_args<T>(L);
  a.skip = FE ? skip : nullptr;
  a.nrhs = nrhs;
  a.inv_nrhs = 1.0 / nrhs;
  a.ld = ld;
  a.u = (const T*)u;
  if (FE && !scratch) scratch = L->scratch();
  a.out = (T*)(FE ? scratch : out);
  a.b = (const T*)b;
  a.xold = (const T*)xold;
  a.sigma = (T)sigma;
  a.theta = (T)theta;
  if (nrhs == 1) {  // tiled order, rows of ceil(Nx / EB) chunks
    a.rowchunks = (a.Nx + C::EB - 1) / C::EB;
    a.tile_y = kTileY;
  }
  if (nrhs > 1 && (nrhs > 64 || L->n_el * nrhs >= ((int64_t)1 << 31)))
    return fail(HMG_ERR_UNSUPPORTED, "several vectors at once: at most 64, and fewer than 2^31 element-vectors");
  const int64_t nb = nrhs == 1 ? (int64_t)a.rowchunks * a.Ny * a.Nz : (L->n_el * nrhs + C::EB - 1) / C::EB;
  if (nb > INT32_MAX / C::WAVES) return fail(HMG_ERR_UNSUPPORTED, "mesh too large for one launch");
  if (!FE && mode == OP_DOT && nrhs > 1) {
    // one partial per work item (element, vector), item e * nrhs + r, into
    // the caller's block (scratch) of n_el * nrhs values: needs groups of one
    // wavefront holding one element
    if (C::EW != 1 || C::GL != 64 || !scratch)
      return fail(HMG_ERR_UNSUPPORTED, "several vectors with u.(A u): degree 6 or 7 and a partials block");
    a.partials = (double*)scratch;
    if (nparts) *nparts = (int)(L->n_el * nrhs);
  } else if (nparts) {  // one partial per wavefront, within the level's partials buffer
    if (nb * C::WAVES > op_partials_capacity(a.Nx, a.Ny, a.Nz))
      return fail(HMG_ERR_WORKSPACE, "operator partial sums exceed their buffer");
    *nparts = (int)nb * C::WAVES;
  }
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
  if (FE) {  // node sums of all vectors in one launch (element-local results n_dg values apart)
    const int64_t Mz = (int64_t)a.Nz * (N - 1) + 1;
    if (Mz * nrhs <= 65535) {
      TRY(fe_node_sum(L, mode, u, out, b, xold, sigma, theta, s, skip, scratch, nrhs, ld));
    } else {  // too many node planes for one grid: vector by vector
      const size_t es = sizeof(T);
      for (int r = 0; r < nrhs; ++r) {
        const size_t o = (size_t)r * ld * es;
        auto at = [&](const void* p) { return p ? (const void*)((const char*)p + o) : nullptr; };
        TRY(fe_node_sum(L, mode, at(u), (char*)out + o, at(b), at(xold), sigma, theta, s, skip,
                        (const char*)scratch + (size_t)r * L->n_dg * es));
      }
    }
  }
  return HMG_OK;
}

template <int N, typename T>
static int dispatch_op(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                       const void* xold, double sigma, double theta, int* nparts, int nrhs, int64_t ld,
                       const int* skip, void* sc, hipStream_t s) {
  const bool curved = L->mesh.curved, fe = L->space == HMG_FE;
  if (curved) {
    if (fe) return run_op<N, T, true, true>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
    return run_op<N, T, true, false>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
  }
  if (fe) return run_op<N, T, false, true>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
  return run_op<N, T, false, false>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
}

template <int N, typename T, bool CURVED, bool P>
static int run_multi_p(int mode, const MultiLaunch& L, hipStream_t s) {
  const MultiArgs<T> m = multi_args<T>(L);
  const dim3 grid(L.grid), block(64 * kOpWaves);
  switch (mode) {
    case OP_APPLY:
      hipLaunchKernelGGL((op_multi_kernel<N, T, CURVED, OP_APPLY, P>), grid, block, 0, s, m);
      break;
    case OP_RESID:
      hipLaunchKernelGGL((op_multi_kernel<N, T, CURVED, OP_RESID, P>), grid, block, 0, s, m);
      break;
    case OP_CHEB:
      hipLaunchKernelGGL((op_multi_kernel<N, T, CURVED, OP_CHEB, P>), grid, block, 0, s, m);
      break;
    default:
      return fail(HMG_ERR_UNSUPPORTED, "multi-mesh launch: apply, residual or Chebyshev");
  }
  return check_launch("op_multi_kernel");
}
template <int N, typename T, bool CURVED>
static int run_multi(int mode, const MultiLaunch& L, hipStream_t s) {
  return L.persist ? run_multi_p<N, T, CURVED, true>(mode, L, s) : run_multi_p<N, T, CURVED, false>(mode, L, s);
}

template <int N, typename T, bool CURVED, bool P>
static int occ_multi_p(int mode) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  constexpr int B = 64 * kOpWaves;
  switch (mode) {
    case OP_APPLY: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_multi_kernel<N, T, CURVED, OP_APPLY, P>, B, 0); break;
    case OP_RESID: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_multi_kernel<N, T, CURVED, OP_RESID, P>, B, 0); break;
    case OP_CHEB: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_multi_kernel<N, T, CURVED, OP_CHEB, P>, B, 0); break;
  }
  return e == hipSuccess ? nb : 0;
}
template <int N, typename T, bool CURVED>
static int occ_multi(int mode) {
  return occ_multi_p<N, T, CURVED, true>(mode);  // persistent grids are sized by this
}

#define HMG_CAT2(a, b) a##b
#define HMG_CAT(a, b) HMG_CAT2(a, b)
#ifdef HMG_ONLY_N
int HMG_CAT(op_launch_n, HMG_ONLY_N)(const hmg_level* L, int mode, const void* u, void* out,
                                      const void* b, const void* xold, double sigma, double theta,
                                      int* nparts, int nrhs, int64_t ld, const int* skip, void* sc,
                                      hipStream_t s) {
  if (L->prec == HMG_F64)
    return dispatch_op<HMG_ONLY_N, double>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
  return dispatch_op<HMG_ONLY_N, float>(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
}
int HMG_CAT(multi_launch_n, HMG_ONLY_N)(int prec, bool curved, int mode, const MultiLaunch& m, hipStream_t s) {
  if (prec == HMG_F64)
    return curved ? run_multi<HMG_ONLY_N, double, true>(mode, m, s) : run_multi<HMG_ONLY_N, double, false>(mode, m, s);
  return curved ? run_multi<HMG_ONLY_N, float, true>(mode, m, s) : run_multi<HMG_ONLY_N, float, false>(mode, m, s);
}
int HMG_CAT(multi_occupancy_n, HMG_ONLY_N)(int prec, bool curved, int mode) {
  if (prec == HMG_F64)
    return curved ? occ_multi<HMG_ONLY_N, double, true>(mode) : occ_multi<HMG_ONLY_N, double, false>(mode);
  return curved ? occ_multi<HMG_ONLY_N, float, true>(mode) : occ_multi<HMG_ONLY_N, float, false>(mode);
}
#endif
#endif  // HMG_DISPATCH_ONLY

#ifdef HMG_DISPATCH_ONLY
#define HMG_DECL(N)                                                                          \
  int op_launch_n##N(const hmg_level*, int, const void*, void*, const void*, const void*,    \
                     double, double, int*, int, int64_t, const int*, void*, hipStream_t);     \
  int multi_launch_n##N(int, bool, int, const MultiLaunch&, hipStream_t);                     \
  int multi_occupancy_n##N(int, bool, int);
HMG_DECL(2)
HMG_DECL(3)
HMG_DECL(4)
HMG_DECL(5)
HMG_DECL(6)
HMG_DECL(7)
HMG_DECL(8)

int launch_operator(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                    const void* xold, double sigma, double theta, int* nparts, hipStream_t s) {
  return launch_operator_batched(L, mode, 1, L->n_dofs, u, out, b, xold, sigma, theta, nparts, s);
}

static int launch_any(const hmg_level* L, int mode, int nrhs, int64_t ld, const void* u, void* out, const void* b,
                      const void* xold, double sigma, double theta, int* nparts, const int* skip, void* sc,
                      hipStream_t s) {
  if (L->n_el == 0 || nrhs == 0) return HMG_OK;
  if (nrhs > 1 && mode == OP_DOT && (L->space != HMG_DG || !sc))
    return fail(HMG_ERR_UNSUPPORTED, "several vectors with u.(A u): DG levels and a partials block only");
  if (nrhs > 1 && L->space != HMG_DG && !sc)
    return fail(HMG_ERR_UNSUPPORTED, "several vectors at once on a continuous FE level need a results block");
  switch (L->n) {
#define HMG_CASE(N) \
  case N: return op_launch_n##N(L, mode, u, out, b, xold, sigma, theta, nparts, nrhs, ld, skip, sc, s);
    HMG_CASE(2) HMG_CASE(3) HMG_CASE(4) HMG_CASE(5) HMG_CASE(6) HMG_CASE(7) HMG_CASE(8)
#undef HMG_CASE
  }
  return fail(HMG_ERR_UNSUPPORTED, "degree must be 1..7");
}

int launch_operator_batched(const hmg_level* L, int mode, int nrhs, int64_t ld, const void* u, void* out,
                            const void* b, const void* xold, double sigma, double theta, int* nparts,
                            hipStream_t s, void* fe_results) {
  return launch_any(L, mode, nrhs, ld, u, out, b, xold, sigma, theta, nparts, nullptr, fe_results, s);
}

int launch_operator_gated(const hmg_level* L, int mode, const void* u, void* out, const void* b,
                          const int* skip, hipStream_t s) {
  return launch_any(L, mode, 1, L->n_dofs, u, out, b, nullptr, 0, 0, nullptr, skip, nullptr, s);
}

int launch_operator_scratch(const hmg_level* L, const void* u, void* out, void* scratch, hipStream_t s) {
  return launch_any(L, OP_APPLY, 1, L->n_dofs, u, out, nullptr, nullptr, 0, 0, nullptr, nullptr, scratch, s);
}

int multi_launch(int n, int prec, bool curved, int mode, const MultiLaunch& m, hipStream_t s) {
  switch (n) {
#define HMG_CASE(N) \
  case N: return multi_launch_n##N(prec, curved, mode, m, s);
    HMG_CASE(2) HMG_CASE(3) HMG_CASE(4) HMG_CASE(5) HMG_CASE(6) HMG_CASE(7) HMG_CASE(8)
#undef HMG_CASE
  }
  return fail(HMG_ERR_UNSUPPORTED, "degree must be 1..7");
}

int multi_occupancy(int n, int prec, bool curved, int mode) {
  switch (n) {
#define HMG_CASE(N) \
  case N: return multi_occupancy_n##N(prec, curved, mode);
    HMG_CASE(2) HMG_CASE(3) HMG_CASE(4) HMG_CASE(5) HMG_CASE(6) HMG_CASE(7) HMG_CASE(8)
#undef HMG_CASE
  }
  return 0;
}

#endif  // HMG_DISPATCH_ONLY

}  // namespace hmg
