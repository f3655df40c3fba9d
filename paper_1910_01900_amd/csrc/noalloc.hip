// Operator apply that allocates nothing and needs no workspace beyond the
// level's own: for callers that cannot allocate device memory at call time
// (work recorded into HIP graphs, tight serving loops, harnesses that forbid
// allocation).  The element-local results of a continuous FE level, which
// hmg_operator_apply keeps in the level's workspace, live here in a static
// device array instead; every call on one GPU shares it.
#include "hmg_internal.h"

#include <mutex>

namespace hmg {
namespace {

constexpr size_t kScratchBytes = HMG_NOALLOC_SCRATCH_BYTES;  // per GPU, held until the process ends
constexpr int kMaxDevices = 64;

// The host name of this array is a stand-in for its device address: every
// host use goes through the pointer hipGetSymbolAddress returns per device.
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_ptr(void** out) {
  int dev = 0;
  HMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HMG_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return HMG_OK;
}

}  // namespace
}  // namespace hmg

using namespace hmg;

extern "C" int hmg_operator_apply_noalloc(const hmg_level* L, const void* u, void* v, hipStream_t s) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  if (!L->bound) return fail(HMG_ERR_WORKSPACE, "level is not bound to a workspace");
  TRY(check_ptr(u, "u"));
  TRY(check_ptr(v, "v"));
  if (u == v) return fail(HMG_ERR_INVALID, "u and v must not overlap");
  const size_t need = L->space == HMG_FE ? (size_t)L->n_dg * L->elem_size() : 0;
  if (need > kScratchBytes)
    return fail(HMG_ERR_UNSUPPORTED, "FE level needs " + std::to_string(need) +
                                         " bytes of element-local results, more than the " +
                                         std::to_string(kScratchBytes) + "-byte static buffer");
  void* p = nullptr;
  if (need) TRY(scratch_ptr(&p));
  return launch_operator_scratch(L, u, v, p, s);
}
