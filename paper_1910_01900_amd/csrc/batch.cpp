// Batches of independent DG meshes of uneven size and degree, several
// right-hand sides each, applied by one launch (all Cartesian meshes, any
// degree) or by one launch per (degree, geometry kind) group; operator,
// residual and the Chebyshev step (the operator fused with the vector
// update) share the schedule.  The schedule -- one launch or one per group,
// persistent workgroups or one per tile, chunks per tile, resident
// workgroups per CU -- is either set by the caller or chosen by timing the
// candidates on the device (hmg_batch_autotune).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <utility>

#include "hmg_internal.h"

using namespace hmg;

namespace {

constexpr int kQs[3] = {1, 2, 4};  // chunks per tile of the three table variants
constexpr int kNq = 3;
constexpr int kMaxChebDeg = 32;
constexpr int kXcd = 8;  // workgroups are dispatched round-robin over 8 XCDs

// One launch of a schedule: the meshes [first, first + count) of the group
// order (all meshes for the single launch).
struct Unit {
  int n = 0;  // nodes per direction (0: mixed, single launch)
  bool curved = false;
  int first = 0, count = 0, group = -1;
  bool persist = false;
  int qi = 0;   // index into kQs
  int bpc = 0;  // resident workgroups per CU (persistent)
  unsigned grid = 0;
  double ms = -1.0;  // time of one launch when chosen by the autotuner
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct hmg_batch {
  std::vector<const hmg_level*> lv;  // batch order (caller-owned levels)
  int prec = HMG_F64, nrhs = 1;
  std::vector<int64_t> off, ld, chunks;  // per mesh (batch order); values, values, workgroup chunks
  int64_t total = 0;                     // values of one packed multi-vector
  std::vector<int> order;                // group order -> batch index
  std::vector<Unit> groups;              // one per (curved, n)
  bool affine = true;
  // tile layout per family (0: single launch, 1: per group) and table variant
  std::vector<int64_t> tile0[2][kNq];  // per mesh, group order
  std::vector<int64_t> xcd[2][kNq];    // family 0: 9 values; family 1: 9 per group
  // workspace
  size_t ws_bytes = 0, off_tab = 0, off_xcd = 0, off_coef = 0, entry = 0;
  char* ws = nullptr;
  bool bound = false;
  int cus = 0;
  // schedule
  bool single = false;
  Unit one;                // the single launch
  std::vector<Unit> sched;  // the per-group launches
  int cheb_deg = 0;
  size_t esize() const { return prec == HMG_F64 ? 8 : 4; }
  int count() const { return (int)lv.size(); }
};

namespace {

// Estimated cost of one workgroup chunk (relative units): items x n^3 x
// (n + 6), curved cells three times the Cartesian work.
double chunk_cost(const hmg_level* L) {
  const double n = L->n;
  return op_elems_per_block(L->n) * n * n * n * (n + 6.0) * (L->mesh.curved ? 3.0 : 1.0);
}

// Split tiles [0, sum T) of meshes with tile counts T[i] and per-tile cost
// c[i] into 8 contiguous ranges of about equal cost.
void split_xcd(const std::vector<int64_t>& T, const std::vector<double>& c, int64_t* x9) {
  double C = 0;
  int64_t tt = 0;
  for (size_t i = 0; i < T.size(); ++i) {
    C += T[i] * c[i];
    tt += T[i];
  }
  x9[0] = 0;
  x9[kXcd] = tt;
  for (int k = 1; k < kXcd; ++k) {
    const double target = C * k / kXcd;
    double acc = 0;
    int64_t tiles = 0, b = tt;
    for (size_t i = 0; i < T.size(); ++i) {
      const double ci = T[i] * c[i];
      if (acc + ci >= target) {
        const int64_t need = (int64_t)std::ceil((target - acc) / c[i]);
        b = tiles + std::min(std::max<int64_t>(need, 0), T[i]);
        break;
      }
      acc += ci;
      tiles += T[i];
    }
    x9[k] = std::max(b, x9[k - 1]);
  }
  for (int k = kXcd - 1; k >= 0; --k) x9[k] = std::min(x9[k], x9[k + 1]);
}

void build_layout(hmg_batch* B) {
  const int cnt = B->count();
  for (int qi = 0; qi < kNq; ++qi) {
    const int q = kQs[qi];
    for (int f = 0; f < 2; ++f) {
      B->tile0[f][qi].assign(cnt, 0);
      B->xcd[f][qi].assign(f == 0 ? 9 : 9 * B->groups.size(), 0);
    }
    // single launch: all meshes, tiles numbered globally
    {
      std::vector<int64_t> T(cnt);
      std::vector<double> c(cnt);
      int64_t t = 0;
      for (int gi = 0; gi < cnt; ++gi) {
        const int m = B->order[gi];
        B->tile0[0][qi][gi] = t;
        T[gi] = (B->chunks[m] + q - 1) / q;
        c[gi] = q * chunk_cost(B->lv[m]);
        t += T[gi];
      }
      split_xcd(T, c, B->xcd[0][qi].data());
    }
    // one launch per group: tiles numbered per group
    for (size_t g = 0; g < B->groups.size(); ++g) {
      const Unit& G = B->groups[g];
      std::vector<int64_t> T(G.count);
      std::vector<double> c(G.count);
      int64_t t = 0;
      for (int j = 0; j < G.count; ++j) {
        const int gi = G.first + j, m = B->order[gi];
        B->tile0[1][qi][gi] = t;
        T[j] = (B->chunks[m] + q - 1) / q;
        c[j] = q * chunk_cost(B->lv[m]);
        t += T[j];
      }
      split_xcd(T, c, B->xcd[1][qi].data() + 9 * g);
    }
  }
}

const int64_t* host_xcd(const hmg_batch* B, int fam, int qi, int group) {
  return B->xcd[fam][qi].data() + (fam == 0 ? 0 : 9 * group);
}
const int64_t* dev_xcd(const hmg_batch* B, int fam, int qi, int group) {
  const int64_t* base = (const int64_t*)(B->ws + B->off_xcd);
  const size_t ng = B->groups.size();
  if (fam == 0) return base + 9 * qi;
  return base + 9 * kNq + 9 * (qi * ng + group);
}

// Grid of a unit: one workgroup per tile of the largest XCD range, or (when
// persistent) at most bpc workgroups per CU.
unsigned unit_grid(const hmg_batch* B, const Unit& U, int fam) {
  const int64_t* x9 = host_xcd(B, fam, U.qi, U.group);
  int64_t mx = 0;
  for (int x = 0; x < kXcd; ++x) mx = std::max(mx, x9[x + 1] - x9[x]);
  int64_t per = mx;
  if (U.persist) per = std::min<int64_t>(mx, (int64_t)U.bpc * ((B->cus + kXcd - 1) / kXcd));
  per = std::max<int64_t>(per, 1);
  if (per > INT32_MAX / kXcd) return 0;  // rejected at launch
  return (unsigned)(per * kXcd);
}

int launch_unit(const hmg_batch* B, const Unit& U, bool single, int mode, hipStream_t s) {
  const int fam = single ? 0 : 1;
  if (U.grid == 0) return fail(HMG_ERR_UNSUPPORTED, "batch too large for one launch");
  MultiLaunch m;
  m.table = B->ws + B->off_tab + ((size_t)(fam * kNq + U.qi) * B->count() + U.first) * B->entry;
  m.count = U.count;
  m.q = kQs[U.qi];
  m.xcd = dev_xcd(B, fam, U.qi, U.group);
  m.grid = U.grid;
  m.persist = U.persist;
  if (single) return fused_launch(B->prec, mode, m, s);
  return multi_launch(U.n, B->prec, U.curved, mode, m, s);
}

int resolve(const hmg_batch* B, int mode, const void* u, void* out, const void* b, const void* xold, int step,
            hipStream_t s) {
  return multi_resolve(B->prec, B->ws + B->off_tab, 2 * kNq * B->count(), u, out, b, xold,
                       mode == OP_CHEB ? B->ws + B->off_coef : nullptr, 2 * kMaxChebDeg, step, s);
}

int run(const hmg_batch* B, int mode, const void* u, void* out, const void* b, const void* xold, int step,
        hipStream_t s) {
  TRY(resolve(B, mode, u, out, b, xold, step, s));
  if (B->single) return launch_unit(B, B->one, true, mode, s);
  for (const Unit& U : B->sched) TRY(launch_unit(B, U, false, mode, s));
  return HMG_OK;
}

template <typename T>
void fill_tables(const hmg_batch* B, std::vector<char>& host) {
  const int cnt = B->count();
  host.assign((size_t)2 * kNq * cnt * sizeof(MeshEntry<T>), 0);
  MeshEntry<T>* E = (MeshEntry<T>*)host.data();
  for (int f = 0; f < 2; ++f)
    for (int qi = 0; qi < kNq; ++qi)
      for (int gi = 0; gi < cnt; ++gi) {
        const int m = B->order[gi];
        const hmg_level* L = B->lv[m];
        MeshEntry<T>& e = E[(size_t)(f * kNq + qi) * cnt + gi];
        e.a = make_args<T>(L);
        e.a.nrhs = B->nrhs;
        e.a.inv_nrhs = 1.0 / B->nrhs;
        e.a.ld = B->ld[m];
        e.off = B->off[m];
        e.tile0 = B->tile0[f][qi][gi];
        e.chunks = B->chunks[m];
        e.n = L->n;
        e.id = m;
      }
}

int check_bound(const hmg_batch* B) {
  if (!B) return fail(HMG_ERR_INVALID, "batch is NULL");
  if (!B->bound) return fail(HMG_ERR_WORKSPACE, "batch is not bound to a workspace");
  return HMG_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char *x = (const char*)a, *y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

int check_vectors(const hmg_batch* B, std::initializer_list<std::pair<const void*, const char*>> in,
                  const void* out) {
  const size_t bytes = (size_t)B->total * B->esize();
  TRY(check_ptr(out, "output"));
  for (auto& p : in) {
    TRY(check_ptr(p.first, p.second));
    if (overlap(p.first, out, bytes)) return fail(HMG_ERR_INVALID, std::string(p.second) + " overlaps the output");
  }
  return HMG_OK;
}

}  // namespace

extern "C" int hmg_batch_create(const hmg_level* const* levels, int count, int nrhs, hmg_batch** out) {
  if (!out) return fail(HMG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!levels || count < 1) return fail(HMG_ERR_INVALID, "need at least one level");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(HMG_ERR_INVALID, "nrhs must be 1..64");
  hmg_batch* B = new hmg_batch;
  B->nrhs = nrhs;
  for (int i = 0; i < count; ++i) {
    const hmg_level* L = levels[i];
    if (!L) {
      delete B;
      return fail(HMG_ERR_INVALID, "level " + std::to_string(i) + " is NULL");
    }
    if (L->space != HMG_DG) {
      delete B;
      return fail(HMG_ERR_UNSUPPORTED, "batches take DG levels only");
    }
    if (i == 0) B->prec = L->prec;
    if (L->prec != B->prec) {
      delete B;
      return fail(HMG_ERR_INVALID, "all levels of a batch must have the same precision");
    }
    const int64_t eb = op_elems_per_block(L->n);
    const int64_t ch = (L->n_el * nrhs + eb - 1) / eb;
    if (ch > INT32_MAX / kOpWaves || L->n_el * nrhs >= ((int64_t)1 << 31)) {
      delete B;
      return fail(HMG_ERR_UNSUPPORTED, "mesh too large for one launch");
    }
    const int64_t per = 256 / (int64_t)L->elem_size();
    const int64_t ld = (L->n_dofs + per - 1) / per * per;  // 256-byte vectors
    B->lv.push_back(L);
    B->off.push_back(B->total);
    B->ld.push_back(ld);
    B->chunks.push_back(ch);
    B->total += ld * nrhs;
    B->affine = B->affine && !L->mesh.curved;
  }
  // group order: Cartesian before curved, ascending degree, batch order inside a group
  std::vector<int> ord(count);
  for (int i = 0; i < count; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const hmg_level *x = B->lv[a], *y = B->lv[b];
    if (x->mesh.curved != y->mesh.curved) return !x->mesh.curved;
    return x->n < y->n;
  });
  B->order = ord;
  for (int gi = 0; gi < count; ++gi) {
    const hmg_level* L = B->lv[ord[gi]];
    if (B->groups.empty() || B->groups.back().n != L->n || B->groups.back().curved != L->mesh.curved) {
      Unit G;
      G.n = L->n;
      G.curved = L->mesh.curved;
      G.first = gi;
      G.group = (int)B->groups.size();
      B->groups.push_back(G);
    }
    B->groups.back().count++;
  }
  build_layout(B);
  B->entry = B->prec == HMG_F64 ? sizeof(MeshEntry<double>) : sizeof(MeshEntry<float>);
  size_t o = 0;
  B->off_tab = o;
  o = align256(o + (size_t)2 * kNq * count * B->entry);
  B->off_xcd = o;
  o = align256(o + sizeof(int64_t) * 9 * kNq * (1 + B->groups.size()));
  B->off_coef = o;
  o = align256(o + (size_t)count * 2 * kMaxChebDeg * B->esize());
  B->ws_bytes = o;
  *out = B;
  return HMG_OK;
}

extern "C" int hmg_batch_query(const hmg_batch* B, int64_t* total_values, size_t* workspace_bytes) {
  if (!B) return fail(HMG_ERR_INVALID, "batch is NULL");
  if (total_values) *total_values = B->total;
  if (workspace_bytes) *workspace_bytes = B->ws_bytes;
  return HMG_OK;
}

extern "C" int hmg_batch_layout(const hmg_batch* B, int i, int64_t* offset, int64_t* ld) {
  if (!B) return fail(HMG_ERR_INVALID, "batch is NULL");
  if (i < 0 || i >= B->count()) return fail(HMG_ERR_INVALID, "mesh index out of range");
  if (offset) *offset = B->off[i];
  if (ld) *ld = B->ld[i];
  return HMG_OK;
}

extern "C" void hmg_batch_destroy(hmg_batch* B) { delete B; }

extern "C" int hmg_batch_bind(hmg_batch* B, void* ws, size_t bytes, hipStream_t s) {
  if (!B) return fail(HMG_ERR_INVALID, "batch is NULL");
  if (!ws || ((uintptr_t)ws & 255)) return fail(HMG_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < B->ws_bytes) return fail(HMG_ERR_WORKSPACE, "workspace too small");
  for (int i = 0; i < B->count(); ++i)
    if (!B->lv[i]->bound) return fail(HMG_ERR_WORKSPACE, "level " + std::to_string(i) + " is not bound");
  int dev = 0;
  HMG_HIP(hipGetDevice(&dev));
  HMG_HIP(hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev));
  B->ws = (char*)ws;
  std::vector<char> tab;
  if (B->prec == HMG_F64) fill_tables<double>(B, tab);
  else fill_tables<float>(B, tab);
  std::vector<int64_t> xc(9 * kNq * (1 + B->groups.size()));
  const size_t ng = B->groups.size();
  for (int qi = 0; qi < kNq; ++qi) {
    std::copy(B->xcd[0][qi].begin(), B->xcd[0][qi].end(), xc.begin() + 9 * qi);
    std::copy(B->xcd[1][qi].begin(), B->xcd[1][qi].end(), xc.begin() + 9 * kNq + 9 * qi * ng);
  }
  std::vector<char> coef((size_t)B->count() * 2 * kMaxChebDeg * B->esize(), 0);
  HMG_HIP(hipMemcpyAsync(B->ws + B->off_tab, tab.data(), tab.size(), hipMemcpyHostToDevice, s));
  HMG_HIP(hipMemcpyAsync(B->ws + B->off_xcd, xc.data(), xc.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  HMG_HIP(hipMemcpyAsync(B->ws + B->off_coef, coef.data(), coef.size(), hipMemcpyHostToDevice, s));
  HMG_HIP(hipStreamSynchronize(s));
  // default schedule: one launch per group, one workgroup per tile of one chunk
  B->single = false;
  B->sched = B->groups;
  for (Unit& U : B->sched) U.grid = unit_grid(B, U, 1);
  B->one = Unit();
  B->one.count = B->count();
  B->one.grid = unit_grid(B, B->one, 0);
  B->cheb_deg = 0;
  B->bound = true;
  return HMG_OK;
}

extern "C" int hmg_batch_set_schedule(hmg_batch* B, int single, int persistent, int chunks_per_tile,
                                      int blocks_per_cu) {
  TRY(check_bound(B));
  int qi = -1;
  for (int i = 0; i < kNq; ++i)
    if (kQs[i] == chunks_per_tile) qi = i;
  if (qi < 0) return fail(HMG_ERR_INVALID, "chunks_per_tile must be 1, 2 or 4");
  if (!persistent && qi != 0) return fail(HMG_ERR_INVALID, "one workgroup per tile needs chunks_per_tile = 1");
  if (persistent && blocks_per_cu < 1) return fail(HMG_ERR_INVALID, "blocks_per_cu must be >= 1");
  if (single && !B->affine) return fail(HMG_ERR_UNSUPPORTED, "the single launch takes Cartesian meshes only");
  auto setu = [&](Unit& U, int fam) {
    U.persist = persistent != 0;
    U.qi = qi;
    U.bpc = persistent ? blocks_per_cu : 0;
    U.grid = unit_grid(B, U, fam);
    U.ms = -1.0;
  };
  B->single = single != 0;
  if (B->single) setu(B->one, 0);
  else
    for (Unit& U : B->sched) setu(U, 1);
  return HMG_OK;
}

extern "C" int hmg_batch_autotune(hmg_batch* B, const void* u, void* v, int reps, hipStream_t s, double* best_ms) {
  TRY(check_bound(B));
  TRY(check_vectors(B, {{u, "u"}}, v));
  if (reps < 1 || reps > 1000) return fail(HMG_ERR_INVALID, "reps must be 1..1000");
  TRY(resolve(B, OP_APPLY, u, v, nullptr, nullptr, 0, s));
  hipEvent_t e0, e1;
  HMG_HIP(hipEventCreate(&e0));
  HMG_HIP(hipEventCreate(&e1));
  int err = HMG_OK;
  // time of one launch of U: best of two rounds of `reps` after two warm-ups
  auto timed = [&](const Unit& U, bool single) -> double {
    for (int w = 0; w < 2 && !err; ++w) err = launch_unit(B, U, single, OP_APPLY, s);
    double best = 1e30;
    for (int r = 0; r < 2 && !err; ++r) {
      if (hipEventRecord(e0, s) != hipSuccess) err = fail(HMG_ERR_HIP, "hipEventRecord");
      for (int i = 0; i < reps && !err; ++i) err = launch_unit(B, U, single, OP_APPLY, s);
      if (!err && hipEventRecord(e1, s) != hipSuccess) err = fail(HMG_ERR_HIP, "hipEventRecord");
      if (!err && hipEventSynchronize(e1) != hipSuccess) err = fail(HMG_ERR_HIP, "hipEventSynchronize");
      float ms = 0;
      if (!err && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) err = fail(HMG_ERR_HIP, "hipEventElapsedTime");
      if (!err) best = std::min(best, (double)ms / reps);
    }
    return best;
  };
  // candidates: one workgroup per tile, or persistent with q in {1, 2, 4}
  // and 1, 2 or the resident maximum of workgroups per CU
  auto tune = [&](Unit& U, bool single) {
    const int fam = single ? 0 : 1;
    const int occ = single ? fused_occupancy(B->prec, OP_APPLY) : multi_occupancy(U.n, B->prec, U.curved, OP_APPLY);
    std::vector<Unit> cand;
    Unit c = U;
    c.persist = false;
    c.qi = 0;
    c.bpc = 0;
    c.grid = unit_grid(B, c, fam);
    const unsigned full = c.grid;
    cand.push_back(c);
    std::vector<int> bpcs = {1, 2};
    if (occ > 2) bpcs.push_back(occ);
    for (int qi = 0; qi < kNq; ++qi)
      for (int bpc : bpcs) {
        if (occ > 0 && bpc > occ) continue;
        Unit p = U;
        p.persist = true;
        p.qi = qi;
        p.bpc = bpc;
        p.grid = unit_grid(B, p, fam);
        if (qi == 0 && p.grid >= full) continue;  // same as one workgroup per tile
        bool dup = false;
        for (const Unit& x : cand)
          if (x.persist && x.qi == p.qi && x.grid == p.grid) dup = true;
        if (!dup) cand.push_back(p);
      }
    double best = 1e30;
    for (const Unit& x : cand) {
      const double t = timed(x, single);
      if (err) return;
      if (t < best) {
        best = t;
        U = x;
        U.ms = t;
      }
    }
  };
  std::vector<Unit> grouped = B->groups;
  double t_grouped = 0;
  for (Unit& U : grouped) {
    tune(U, false);
    if (err) break;
    t_grouped += U.ms;
  }
  Unit one = B->one;
  double t_one = 1e30;
  if (!err && B->affine) {
    tune(one, true);
    if (!err) t_one = one.ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err) return err;
  B->sched = grouped;
  B->one = one;
  B->single = t_one < t_grouped;
  if (best_ms) *best_ms = std::min(t_one, t_grouped);
  return HMG_OK;
}

extern "C" int hmg_batch_schedule(const hmg_batch* B, int* single, int* units) {
  TRY(check_bound(B));
  if (single) *single = B->single ? 1 : 0;
  if (units) *units = B->single ? 1 : (int)B->sched.size();
  return HMG_OK;
}

extern "C" int hmg_batch_unit_info(const hmg_batch* B, int u, int* n, int* curved, int* meshes, int* persistent,
                                   int* chunks_per_tile, int* blocks_per_cu, unsigned* grid, double* ms) {
  TRY(check_bound(B));
  const int nu = B->single ? 1 : (int)B->sched.size();
  if (u < 0 || u >= nu) return fail(HMG_ERR_INVALID, "unit index out of range");
  const Unit& U = B->single ? B->one : B->sched[u];
  if (n) *n = U.n;
  if (curved) *curved = U.curved ? 1 : 0;
  if (meshes) *meshes = U.count;
  if (persistent) *persistent = U.persist ? 1 : 0;
  if (chunks_per_tile) *chunks_per_tile = kQs[U.qi];
  if (blocks_per_cu) *blocks_per_cu = U.bpc;
  if (grid) *grid = U.grid;
  if (ms) *ms = U.ms;
  return HMG_OK;
}

extern "C" int hmg_batch_apply(const hmg_batch* B, const void* u, void* v, hipStream_t s) {
  TRY(check_bound(B));
  TRY(check_vectors(B, {{u, "u"}}, v));
  return run(B, OP_APPLY, u, v, nullptr, nullptr, 0, s);
}

extern "C" int hmg_batch_residual(const hmg_batch* B, const void* b, const void* u, void* r, hipStream_t s) {
  TRY(check_bound(B));
  TRY(check_vectors(B, {{u, "u"}}, r));
  TRY(check_ptr(b, "b"));
  return run(B, OP_RESID, u, r, b, nullptr, 0, s);
}

extern "C" int hmg_batch_set_chebyshev(hmg_batch* B, const double* lmax, int degree, double lof, double hif,
                                       hipStream_t s) {
  TRY(check_bound(B));
  if (!lmax) return fail(HMG_ERR_INVALID, "lmax is NULL");
  if (degree < 1 || degree > kMaxChebDeg) return fail(HMG_ERR_INVALID, "degree must be 1..32");
  if (!(lof > 0) || !(hif > lof)) return fail(HMG_ERR_INVALID, "need 0 < lo_frac < hi_frac");
  const int cnt = B->count();
  std::vector<double> c((size_t)cnt * 2 * kMaxChebDeg, 0.0);
  for (int m = 0; m < cnt; ++m) {
    if (!(lmax[m] > 0) || !std::isfinite(lmax[m])) return fail(HMG_ERR_INVALID, "lmax must be positive and finite");
    std::vector<double> sig, th;
    cheb_coeffs(degree, lmax[m], lof, hif, sig, th);
    for (int j = 0; j < degree; ++j) {
      c[(size_t)m * 2 * kMaxChebDeg + 2 * j] = j == 0 ? 0.0 : sig[j];
      c[(size_t)m * 2 * kMaxChebDeg + 2 * j + 1] = th[j];
    }
  }
  if (B->prec == HMG_F64) {
    HMG_HIP(hipMemcpyAsync(B->ws + B->off_coef, c.data(), c.size() * 8, hipMemcpyHostToDevice, s));
    HMG_HIP(hipStreamSynchronize(s));
  } else {
    std::vector<float> f(c.begin(), c.end());
    HMG_HIP(hipMemcpyAsync(B->ws + B->off_coef, f.data(), f.size() * 4, hipMemcpyHostToDevice, s));
    HMG_HIP(hipStreamSynchronize(s));
  }
  B->cheb_deg = degree;
  return HMG_OK;
}

// Alg. 3 on every mesh and vector of the batch with the result left in x
// (x holds the start vector); tmp is a second packed vector.
extern "C" int hmg_batch_chebyshev_smooth(const hmg_batch* B, const void* b, void* x, void* tmp, hipStream_t s) {
  TRY(check_bound(B));
  if (B->cheb_deg < 1) return fail(HMG_ERR_INVALID, "Chebyshev coefficients not set");
  TRY(check_vectors(B, {{b, "b"}, {tmp, "tmp"}}, x));
  if (overlap(b, tmp, (size_t)B->total * B->esize())) return fail(HMG_ERR_INVALID, "b overlaps tmp");
  const int ns = B->cheb_deg;
  void *cur, *oth;
  if ((ns & 1) == 0) {
    cur = x;
    oth = tmp;
  } else {
    TRY(vec_copy(B->prec, x, tmp, B->total, s));
    cur = tmp;
    oth = x;
  }
  TRY(run(B, OP_CHEB, cur, oth, b, cur, 0, s));
  std::swap(cur, oth);
  for (int j = 1; j < ns; ++j) {
    TRY(run(B, OP_CHEB, cur, oth, b, oth, j, s));
    std::swap(cur, oth);
  }
  if (cur != x) return fail(HMG_ERR_INVALID, "internal: Chebyshev buffer parity");
  return HMG_OK;
}
