// Multi-mesh operator launch over Cartesian DG meshes of any degree in ONE
// kernel: each tile dispatches on its mesh's degree to the operator body of
// that degree (op_body.h).  The workgroup's LDS is sized for the largest
// degree, so residency is that of the largest degree for every tile; the
// batch scheduler weighs this against one launch per degree by timing both.
#include "op_body.h"

namespace hmg {

template <int N>
constexpr int fused_block_lds() {  // a workgroup's LDS at degree N, the larger precision (in values)
  using C = Cfg<N, false, false>;
  return C::GROUPS * (op_group_lds<N, float, false, false, OP_CHEB>() > op_group_lds<N, double, false, false, OP_CHEB>()
                          ? op_group_lds<N, float, false, false, OP_CHEB>()
                          : op_group_lds<N, double, false, false, OP_CHEB>());
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kFusedBlock =
    cmax(cmax(cmax(fused_block_lds<2>(), fused_block_lds<3>()), cmax(fused_block_lds<4>(), fused_block_lds<5>())),
         cmax(cmax(fused_block_lds<6>(), fused_block_lds<7>()), fused_block_lds<8>()));

// One tile of mesh E (degree N): the lane tables of that degree into the
// group's LDS, then its chunks.  The groups of consecutive tiles of
// different degrees overlap in LDS: a workgroup barrier first.
template <int N, typename T, int MODE, bool PERSIST>
__device__ __forceinline__ void fused_tile(const MultiArgs<T>& m, cptr<MeshEntry<T>> E, int64_t tile, T* smem) {
  using C = Cfg<N, false, false>;
  constexpr int WL = op_group_lds<N, T, false, false, MODE>();
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / C::GL);  // group-uniform (scalar)
  T* const W0 = smem + grp * WL;
  __syncthreads();  // the previous tile's LDS reads come first
  load_lane_tables<T, C::LT, C::GL>(E->a.tabs, W0 + C::EW * C::PER);
  if constexpr (PERSIST) {
    multi_tile<N, T, false, MODE>(m, E, tile, W0);
  } else {
    const OpArgs<T>& a = *(const OpArgs<T>*)&E->a;
    const int64_t it0 = (tile - E->tile0) * C::EB + (int64_t)grp * C::EW;
    op_items<N, T, false, false, MODE>(a, it0, group_count(a, it0), W0);
  }
}

template <typename T, int MODE, bool PERSIST>
__device__ __forceinline__ void fused_switch(const MultiArgs<T>& m, cptr<MeshEntry<T>> E, int64_t tile, T* W0) {
  switch (E->n) {
    case 2: fused_tile<2, T, MODE, PERSIST>(m, E, tile, W0); break;
    case 3: fused_tile<3, T, MODE, PERSIST>(m, E, tile, W0); break;
    case 4: fused_tile<4, T, MODE, PERSIST>(m, E, tile, W0); break;
    case 5: fused_tile<5, T, MODE, PERSIST>(m, E, tile, W0); break;
    case 6: fused_tile<6, T, MODE, PERSIST>(m, E, tile, W0); break;
    case 7: fused_tile<7, T, MODE, PERSIST>(m, E, tile, W0); break;
    default: fused_tile<8, T, MODE, PERSIST>(m, E, tile, W0); break;
  }
}

// Tiles as in the per-degree multi-mesh kernel: XCD x takes the contiguous
// range [xcd[x], xcd[x+1]); PERSIST: its workgroups stride through it,
// otherwise one workgroup per tile of one chunk.
template <typename T, int MODE, bool PERSIST>
__global__ void __launch_bounds__(256) op_fused_kernel(const MultiArgs<T> m) {
  __shared__ T smem[kFusedBlock];
  T* const W0 = smem;  // each tile places its groups in it
  const cptr<MeshEntry<T>> tab = (cptr<MeshEntry<T>>)(uintptr_t)m.table;
  const cptr<int64_t> xcd = (cptr<int64_t>)(uintptr_t)m.xcd;
  const int x = blockIdx.x & 7;
  const int64_t end = xcd[x + 1];
  int64_t tile = xcd[x] + (blockIdx.x >> 3);
  if (tile >= end) return;
  int mi = find_mesh(tab, m.count, tile);
  if constexpr (PERSIST) {
    const int64_t stride = gridDim.x >> 3;
    for (; tile < end; tile += stride) {
      while (mi + 1 < m.count && tab[mi + 1].tile0 <= tile) ++mi;
      fused_switch<T, MODE, true>(m, tab + mi, tile, W0);
    }
  } else {
    fused_switch<T, MODE, false>(m, tab + mi, tile, W0);
  }
}

template <typename T, bool P>
static int run_fused_p(int mode, const MultiLaunch& L, hipStream_t s) {
  const MultiArgs<T> m = multi_args<T>(L);
  const dim3 grid(L.grid), block(64 * kOpWaves);
  switch (mode) {
    case OP_APPLY: hipLaunchKernelGGL((op_fused_kernel<T, OP_APPLY, P>), grid, block, 0, s, m); break;
    case OP_RESID: hipLaunchKernelGGL((op_fused_kernel<T, OP_RESID, P>), grid, block, 0, s, m); break;
    case OP_CHEB: hipLaunchKernelGGL((op_fused_kernel<T, OP_CHEB, P>), grid, block, 0, s, m); break;
    default: return fail(HMG_ERR_UNSUPPORTED, "multi-mesh launch: apply, residual or Chebyshev");
  }
  return check_launch("op_fused_kernel");
}
template <typename T>
static int run_fused(int mode, const MultiLaunch& L, hipStream_t s) {
  return L.persist ? run_fused_p<T, true>(mode, L, s) : run_fused_p<T, false>(mode, L, s);
}

template <typename T>
static int occ_fused(int mode) {  // persistent grids are sized by this
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  constexpr int B = 64 * kOpWaves;
  switch (mode) {
    case OP_APPLY: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_fused_kernel<T, OP_APPLY, true>, B, 0); break;
    case OP_RESID: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_fused_kernel<T, OP_RESID, true>, B, 0); break;
    case OP_CHEB: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, op_fused_kernel<T, OP_CHEB, true>, B, 0); break;
  }
  return e == hipSuccess ? nb : 0;
}

// ------------------------------------------------------------------ resolve
template <typename T>
__global__ void k_multi_resolve(MeshEntry<T>* table, int count, const T* u, T* out, const T* b, const T* xold,
                                const T* coef, int cstride, int step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  MeshEntry<T>& E = table[i];
  const int64_t off = E.off;
  E.a.u = u + off;
  E.a.out = out + off;
  E.a.b = b ? b + off : nullptr;
  E.a.xold = xold ? xold + off : nullptr;
  if (coef) {
    E.a.sigma = coef[(int64_t)E.id * cstride + 2 * step];
    E.a.theta = coef[(int64_t)E.id * cstride + 2 * step + 1];
  }
}

int multi_resolve(int prec, void* table, int count, const void* u, void* out, const void* b, const void* xold,
                  const void* coef, int cstride, int step, hipStream_t s) {
  if (count <= 0) return HMG_OK;
  const unsigned g = (unsigned)((count + 63) / 64);
  if (prec == HMG_F64)
    hipLaunchKernelGGL(k_multi_resolve<double>, g, 64, 0, s, (MeshEntry<double>*)table, count, (const double*)u,
                       (double*)out, (const double*)b, (const double*)xold, (const double*)coef, cstride, step);
  else
    hipLaunchKernelGGL(k_multi_resolve<float>, g, 64, 0, s, (MeshEntry<float>*)table, count, (const float*)u,
                       (float*)out, (const float*)b, (const float*)xold, (const float*)coef, cstride, step);
  return check_launch("multi_resolve");
}

int fused_launch(int prec, int mode, const MultiLaunch& m, hipStream_t s) {
  return prec == HMG_F64 ? run_fused<double>(mode, m, s) : run_fused<float>(mode, m, s);
}
int fused_occupancy(int prec, int mode) { return prec == HMG_F64 ? occ_fused<double>(mode) : occ_fused<float>(mode); }

}  // namespace hmg
