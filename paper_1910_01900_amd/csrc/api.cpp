// C ABI: handles, workspace layout, smoother / transfer / V-cycle / PCG
// drivers (Alg. 1-3) and the coarse-level exact solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "net_internal.h"

namespace hmg {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}
int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HMG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return HMG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int to_mesh(const hmg_mesh_desc* d, Mesh& m) {
  if (!d) return fail(HMG_ERR_INVALID, "mesh descriptor is NULL");
  for (int r = 0; r < 3; ++r) {
    if (d->nel[r] < 1) return fail(HMG_ERR_INVALID, "nel must be >= 1");
    if (!(d->hi[r] > d->lo[r])) return fail(HMG_ERR_INVALID, "hi must exceed lo");
    m.N[r] = d->nel[r];
    m.lo[r] = d->lo[r];
    m.hi[r] = d->hi[r];
  }
  if (d->degree < 1 || d->degree > 7) return fail(HMG_ERR_UNSUPPORTED, "degree must be 1..7");
  m.k = d->degree;
  m.curved = d->deformed != 0;
  m.amp = d->deform_amp;
  m.waves = d->deform_waves < 1 ? 1 : d->deform_waves;
  if (d->mapping_degree != 0 && d->mapping_degree != 3)
    return fail(HMG_ERR_UNSUPPORTED, "mapping_degree must be 3 (cubic) or 0 (exact)");
  m.mapdeg = d->mapping_degree;
  for (int f = 0; f < 6; ++f) {
    if (d->bc[f] > 1) return fail(HMG_ERR_INVALID, "bc must be 0 (Dirichlet) or 1 (Neumann)");
    m.bc[f] = d->bc[f];
  }
  m.ip = d->ip_factor > 0 ? d->ip_factor : 1.0;
  const int64_t ne = m.n_el();
  if (ne > ((int64_t)1 << 31)) return fail(HMG_ERR_UNSUPPORTED, "too many elements");
  m.tau_scale.clear();
  if (d->tau_scale) m.tau_scale.assign(d->tau_scale, d->tau_scale + ne);
  return HMG_OK;
}

int check_ptr(const void* p, const char* what) {
  if (!p) return fail(HMG_ERR_INVALID, std::string(what) + " is NULL");
  if (((uintptr_t)p) & 255) return fail(HMG_ERR_INVALID, std::string(what) + " is not 256-byte aligned");
  return HMG_OK;
}

// ------------------------------------------------------------------ dense Cholesky
// In-place lower Cholesky (row-major), blocked, trailing updates threaded.
static bool cholesky(std::vector<double>& A, int n) {
  const int bs = 64;
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  for (int k0 = 0; k0 < n; k0 += bs) {
    const int k1 = std::min(n, k0 + bs);
    for (int j = k0; j < k1; ++j) {
      double d = A[(size_t)j * n + j];
      for (int k = k0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
      if (!(d > 0)) return false;
      d = std::sqrt(d);
      A[(size_t)j * n + j] = d;
      for (int i = j + 1; i < k1; ++i) {
        double s = A[(size_t)i * n + j];
        for (int k = k0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
        A[(size_t)i * n + j] = s / d;
      }
    }
    auto panel = [&](int ia, int ib) {
      for (int i = ia; i < ib; ++i) {
        double* Ai = &A[(size_t)i * n];
        for (int j = k0; j < k1; ++j) {
          double s = Ai[j];
          const double* Aj = &A[(size_t)j * n];
          for (int k = k0; k < j; ++k) s -= Ai[k] * Aj[k];
          Ai[j] = s / Aj[j];
        }
        for (int j = k1; j <= i; ++j) {
          const double* Aj = &A[(size_t)j * n];
          double s = 0.0;
          for (int k = k0; k < k1; ++k) s += Ai[k] * Aj[k];
          Ai[j] -= s;
        }
      }
    };
    // panel rows first (they are read by the trailing update of later rows)
    std::vector<std::thread> th;
    auto par = [&](auto fn, int a, int b) {
      th.clear();
      int chunk = (b - a + (int)nt - 1) / (int)nt;
      for (unsigned t = 0; t < nt; ++t) {
        int x = a + (int)t * chunk, y = std::min(b, x + chunk);
        if (x >= y) break;
        th.emplace_back(fn, x, y);
      }
      for (auto& t : th) t.join();
    };
    // triangular solve of the panel, then trailing update
    par([&](int ia, int ib) {
      for (int i = ia; i < ib; ++i) {
        double* Ai = &A[(size_t)i * n];
        for (int j = k0; j < k1; ++j) {
          double s = Ai[j];
          const double* Aj = &A[(size_t)j * n];
          for (int k = k0; k < j; ++k) s -= Ai[k] * Aj[k];
          Ai[j] = s / Aj[j];
        }
      }
    }, k1, n);
    par([&](int ia, int ib) {
      for (int i = ia; i < ib; ++i) {
        double* Ai = &A[(size_t)i * n];
        for (int j = k1; j <= i; ++j) {
          const double* Aj = &A[(size_t)j * n];
          double s = 0.0;
          for (int k = k0; k < k1; ++k) s += Ai[k] * Aj[k];
          Ai[j] -= s;
        }
      }
    }, k1, n);
    (void)panel;
  }
  return true;
}

// A^{-1} = L^{-T} L^{-1} from the Cholesky factor (row-major, lower).
static void chol_inverse(const std::vector<double>& L, int n, std::vector<double>& Ainv) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<double> W((size_t)n * n, 0.0);  // W[j][i] = (L^{-1})[i][j], i >= j
  auto run = [&](auto fn) {
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(fn, (int)t);
    for (auto& t : th) t.join();
  };
  run([&](int t) {
    for (int j = t; j < n; j += (int)nt) {
      double* y = &W[(size_t)j * n];
      for (int i = j; i < n; ++i) {
        const double* Li = &L[(size_t)i * n];
        double s = (i == j) ? 1.0 : 0.0;
        for (int k = j; k < i; ++k) s -= Li[k] * y[k];
        y[i] = s / Li[i];
      }
    }
  });
  Ainv.assign((size_t)n * n, 0.0);
  run([&](int t) {
    for (int i = t; i < n; i += (int)nt)
      for (int j = 0; j <= i; ++j) {
        const double* a = &W[(size_t)i * n];
        const double* b = &W[(size_t)j * n];
        double s = 0.0;
        for (int k = i; k < n; ++k) s += a[k] * b[k];
        Ainv[(size_t)i * n + j] = s;
        Ainv[(size_t)j * n + i] = s;
      }
  });
}

// largest eigenvalue of a symmetric tridiagonal matrix by Sturm bisection
static double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0) + (i + 1 < m ? std::fabs(b[i]) : 0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m) hi = mid;
    else lo = mid;
    if (hi - lo <= 1e-15 * std::fabs(hi)) break;
  }
  return hi;
}

// Classical Chebyshev iteration coefficients (Saad, Alg. 12.1) on [lo, hi]*lmax.
void cheb_coeffs(int ns, double lmax, double lof, double hif, std::vector<double>& sig,
                        std::vector<double>& th) {
  const double a = lof * lmax, b = hif * lmax;
  const double c = 0.5 * (b + a), delta = 0.5 * (b - a), s1 = c / delta;
  sig.assign(ns, 0.0);
  th.assign(ns, 0.0);
  th[0] = 1.0 / c;
  double rho_prev = 1.0 / s1;
  for (int j = 1; j < ns; ++j) {
    const double rho = 1.0 / (2.0 * s1 - rho_prev);
    sig[j] = rho * rho_prev;
    th[j] = 2.0 * rho / delta;
    rho_prev = rho;
  }
}

}  // namespace hmg

using namespace hmg;

extern "C" const char* hmg_last_error(void) { return g_err.c_str(); }
extern "C" int hmg_version(void) { return 400; }

// ================================================================== levels
static int level_init(const Mesh& m, int space, int prec, hmg_level** out) {
  if (space != HMG_DG && space != HMG_FE) return fail(HMG_ERR_INVALID, "space must be DG or FE");
  if (prec != HMG_F64 && prec != HMG_F32) return fail(HMG_ERR_INVALID, "prec must be F64 or F32");
  hmg_level* L = new hmg_level();
  L->mesh = m;
  L->space = space;
  L->prec = prec;
  L->k = m.k;
  L->n = m.k + 1;
  L->n_el = m.n_el();
  L->n_dg = L->n_el * L->n * L->n * L->n;
  L->n_dofs = space == HMG_DG ? L->n_dg
                              : ((int64_t)m.N[0] * m.k + 1) * ((int64_t)m.N[1] * m.k + 1) *
                                    ((int64_t)m.N[2] * m.k + 1);
  L->basis = make_basis(m.k);
  int rc = build_geometry(m, L->basis, L->geom, space == HMG_DG);
  if (rc) {
    delete L;
    return rc;
  }
  rc = diag_host(m, L->basis, L->geom, space, L->diag_h);
  if (rc) {
    delete L;
    return rc;
  }
  if (space == HMG_FE)
    for (int d = 0; d < 3; ++d) L->geom.face[d].clear();
  // workspace layout
  const size_t es = L->elem_size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  L->off_metric = take(L->geom.metric.size() * es);
  for (int d = 0; d < 3; ++d) L->off_face[d] = take(L->geom.face[d].size() * es);
  L->off_tau = take((size_t)L->n_el * es);
  L->off_diag = take(L->vec_bytes());
  L->off_dinv = take(L->vec_bytes());
  L->off_tmp = take((size_t)kTmpVecs * L->vec_bytes());
  L->off_scratch = take(space == HMG_FE ? (size_t)L->n_dg * es : 0);
  L->off_part = take((size_t)op_partials_capacity(L->mesh.N[0], L->mesh.N[1], L->mesh.N[2]) * 8);
  L->off_scal = take(16 * 8);
  L->off_tabs = take((size_t)TabOff(L->n).size() * es);
  L->ws_bytes = off;
  *out = L;
  return HMG_OK;
}

extern "C" int hmg_level_create(const hmg_mesh_desc* desc, int space, int prec, hmg_level** out) {
  if (!out) return fail(HMG_ERR_INVALID, "out is NULL");
  Mesh m;
  TRY(to_mesh(desc, m));
  return level_init(m, space, prec, out);
}

extern "C" int hmg_level_query(const hmg_level* L, int64_t* n_dofs, size_t* ws) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  if (n_dofs) *n_dofs = L->n_dofs;
  if (ws) *ws = L->ws_bytes;
  return HMG_OK;
}

template <typename T>
static int upload(const std::vector<double>& h, void* dst, hipStream_t s, std::vector<char>& keep) {
  if (h.empty()) return HMG_OK;
  const size_t bytes = h.size() * sizeof(T);
  std::vector<char> buf(bytes);
  T* p = (T*)buf.data();
  for (size_t i = 0; i < h.size(); ++i) p[i] = (T)h[i];
  HMG_HIP(hipMemcpyAsync(dst, buf.data(), bytes, hipMemcpyHostToDevice, s));
  HMG_HIP(hipStreamSynchronize(s));
  (void)keep;
  return HMG_OK;
}

extern "C" int hmg_level_bind(hmg_level* L, void* ws, size_t bytes, hipStream_t s) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  if (!ws || (((uintptr_t)ws) & 255)) return fail(HMG_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < L->ws_bytes) return fail(HMG_ERR_WORKSPACE, "workspace too small");
  L->ws = (char*)ws;
  std::vector<char> keep;
  const Geometry& g = L->geom;
  if (L->prec == HMG_F64) {
    TRY(upload<double>(g.metric, L->metric(), s, keep));
    for (int d = 0; d < 3; ++d) TRY(upload<double>(g.face[d], L->face(d), s, keep));
    TRY(upload<double>(g.tau, L->tau(), s, keep));
  } else {
    TRY(upload<float>(g.metric, L->metric(), s, keep));
    for (int d = 0; d < 3; ++d) TRY(upload<float>(g.face[d], L->face(d), s, keep));
    TRY(upload<float>(g.tau, L->tau(), s, keep));
  }
  {
    const std::vector<double> tabs = op_tables(L->basis);
    if (L->prec == HMG_F64) {
      TRY(upload<double>(tabs, L->tabs(), s, keep));
    } else {
      TRY(upload<float>(tabs, L->tabs(), s, keep));
    }
  }
  // diagonal (computed during create) and its inverse
  const std::vector<double>& dg = L->diag_h;
  std::vector<double> di(dg.size());
  for (size_t i = 0; i < dg.size(); ++i) di[i] = 1.0 / dg[i];
  if (L->prec == HMG_F64) {
    TRY(upload<double>(dg, L->diag(), s, keep));
    TRY(upload<double>(di, L->dinv(), s, keep));
  } else {
    TRY(upload<float>(dg, L->diag(), s, keep));
    TRY(upload<float>(di, L->dinv(), s, keep));
  }
  L->bound = true;
  L->geom.metric.clear();
  L->geom.metric.shrink_to_fit();
  for (int d = 0; d < 3; ++d) {
    L->geom.face[d].clear();
    L->geom.face[d].shrink_to_fit();
  }
  return HMG_OK;
}

extern "C" void hmg_level_destroy(hmg_level* L) { delete L; }

static int check_level(const hmg_level* L) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  if (!L->bound) return fail(HMG_ERR_WORKSPACE, "level is not bound to a workspace");
  return HMG_OK;
}

extern "C" int hmg_operator_apply(const hmg_level* L, const void* u, void* v, hipStream_t s) {
  TRY(check_level(L));
  TRY(check_ptr(u, "u"));
  TRY(check_ptr(v, "v"));
  if (u == v) return fail(HMG_ERR_INVALID, "u and v must not overlap");
  return launch_operator(L, OP_APPLY, u, v, nullptr, nullptr, 0, 0, nullptr, s);
}

extern "C" int hmg_residual(const hmg_level* L, const void* b, const void* u, void* r, hipStream_t s) {
  TRY(check_level(L));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(u, "u"));
  TRY(check_ptr(r, "r"));
  if (u == r) return fail(HMG_ERR_INVALID, "u and r must not overlap");
  return launch_operator(L, OP_RESID, u, r, b, nullptr, 0, 0, nullptr, s);
}

static int check_batch(const hmg_level* L, int nrhs, int64_t ld) {
  if (L->space != HMG_DG) return fail(HMG_ERR_UNSUPPORTED, "several vectors at once: DG levels only");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(HMG_ERR_INVALID, "nrhs must be 1..64");
  if (ld < L->n_dofs) return fail(HMG_ERR_INVALID, "ld must be at least the level's DoF count");
  if ((ld * (int64_t)L->elem_size()) % 256) return fail(HMG_ERR_INVALID, "ld * element size must be a multiple of 256 bytes");
  return HMG_OK;
}

static bool ranges_overlap(const void* a, const void* b, size_t bytes) {
  const char *x = (const char*)a, *y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

extern "C" int hmg_operator_apply_batched(const hmg_level* L, int nrhs, const void* u, void* v, int64_t ld,
                                          hipStream_t s) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  TRY(check_batch(L, nrhs, ld));
  TRY(check_level(L));
  TRY(check_ptr(u, "u"));
  TRY(check_ptr(v, "v"));
  if (ranges_overlap(u, v, (size_t)(ld * (nrhs - 1) + L->n_dofs) * L->elem_size()))
    return fail(HMG_ERR_INVALID, "u and v must not overlap");
  return launch_operator_batched(L, OP_APPLY, nrhs, ld, u, v, nullptr, nullptr, 0, 0, nullptr, s);
}

extern "C" int hmg_residual_batched(const hmg_level* L, int nrhs, const void* b, const void* u, void* r,
                                    int64_t ld, hipStream_t s) {
  if (!L) return fail(HMG_ERR_INVALID, "level is NULL");
  TRY(check_batch(L, nrhs, ld));
  TRY(check_level(L));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(u, "u"));
  TRY(check_ptr(r, "r"));
  if (ranges_overlap(u, r, (size_t)(ld * (nrhs - 1) + L->n_dofs) * L->elem_size()))
    return fail(HMG_ERR_INVALID, "u and r must not overlap");
  return launch_operator_batched(L, OP_RESID, nrhs, ld, u, r, b, nullptr, 0, 0, nullptr, s);
}

extern "C" int hmg_level_diagonal_host(const hmg_level* L, double* out) {
  if (!L || !out) return fail(HMG_ERR_INVALID, "NULL argument");
  std::copy(L->diag_h.begin(), L->diag_h.end(), out);
  return HMG_OK;
}

extern "C" int hmg_diagonal(const hmg_level* L, void* d, hipStream_t s) {
  TRY(check_level(L));
  TRY(check_ptr(d, "d"));
  return vec_copy(L->prec, L->diag(), d, L->n_dofs, s);
}

static int estimate_lmax(const hmg_level* L, int iters, uint64_t seed, double* lmax, hipStream_t s) {
  const int pr = L->prec;
  const int64_t n = L->n_dofs;
  void *r = L->tmp(0), *z = L->tmp(1), *p = L->tmp(2), *Ap = L->tmp(3);
  double* scal = L->scal();
  double* part = L->partials();
  TRY(vec_splitmix(pr, seed, r, n, s));
  TRY(vec_mul3(pr, 1.0, L->dinv(), r, z, n, s));
  TRY(vec_copy(pr, z, p, n, s));
  TRY(vec_dot(pr, r, z, n, part, scal + 0, s));
  double rz;
  HMG_HIP(hipMemcpyAsync(&rz, scal + 0, 8, hipMemcpyDeviceToHost, s));
  HMG_HIP(hipStreamSynchronize(s));
  std::vector<double> alpha, beta;
  for (int it = 0; it < iters; ++it) {
    TRY(launch_operator(L, OP_APPLY, p, Ap, nullptr, nullptr, 0, 0, nullptr, s));
    TRY(vec_dot(pr, p, Ap, n, part, scal + 1, s));
    double pAp;
    HMG_HIP(hipMemcpyAsync(&pAp, scal + 1, 8, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    if (!(pAp > 0) || !(rz > 0)) break;
    const double a = rz / pAp;
    TRY(vec_axpby(pr, 1.0, r, -a, Ap, r, n, s));
    TRY(vec_mul3(pr, 1.0, L->dinv(), r, z, n, s));
    TRY(vec_dot(pr, r, z, n, part, scal + 0, s));
    double rzn;
    HMG_HIP(hipMemcpyAsync(&rzn, scal + 0, 8, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    const double bta = rzn / rz;
    alpha.push_back(a);
    beta.push_back(bta);
    rz = rzn;
    TRY(vec_axpby(pr, 1.0, z, bta, p, p, n, s));
    if (!(rzn > 0)) break;
  }
  const int m = (int)alpha.size();
  if (m == 0) return fail(HMG_ERR_BREAKDOWN, "lambda_max: CG broke down at the first step");
  std::vector<double> da(m), ob(std::max(0, m - 1));
  for (int j = 0; j < m; ++j) {
    da[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < m) ob[j] = std::sqrt(beta[j]) / alpha[j];
  }
  *lmax = tridiag_max_eig(da, ob);
  return HMG_OK;
}

extern "C" int hmg_estimate_lambda_max(const hmg_level* L, int iters, uint64_t seed, double* lmax,
                                       hipStream_t s) {
  TRY(check_level(L));
  if (!lmax || iters < 1) return fail(HMG_ERR_INVALID, "lmax NULL or iters < 1");
  return estimate_lmax(L, iters, seed, lmax, s);
}

// Alg. 3 with the result left in x; uses tmp(0) as the second buffer.
static int chebyshev(const hmg_level* L, const void* b, void* x, int ns, double lmax, double lof,
                     double hif, int x_is_zero, hipStream_t s) {
  std::vector<double> sig, th;
  cheb_coeffs(ns, lmax, lof, hif, sig, th);
  const int pr = L->prec;
  const int64_t n = L->n_dofs;
  void* tmp = L->tmp(0);
  void *cur, *oth;
  bool x0_zero = false;
  if (!x_is_zero && (ns & 1) && ns >= 3) {
    // odd degree from a nonzero start without copying x: iterates 1, 3, ..
    // go to tmp and 2, 4, .. back to x, iterate ns - 1 to tmp(1), the last to x
    // (each step writes a buffer other than its input; out may alias x_old)
    void* const tmp2 = L->tmp(1);
    void *prev = x, *at = x;
    for (int j = 0; j < ns; ++j) {
      void* out = j == ns - 1 ? x : (j == ns - 2 ? tmp2 : ((j & 1) ? x : tmp));
      TRY(launch_operator(L, OP_CHEB, at, out, b, j == 0 ? at : prev, j == 0 ? 0.0 : sig[j], th[j], nullptr, s));
      prev = at;
      at = out;
    }
    return HMG_OK;
  }
  if (x_is_zero) {
    // x_1 = theta_0 D^{-1} b, x_0 = 0; ns-1 swaps follow
    if (((ns - 1) & 1) == 0) {
      cur = x;
      oth = tmp;
    } else {
      cur = tmp;
      oth = x;
    }
    TRY(vec_mul3(pr, th[0], L->dinv(), b, cur, n, s));
    x0_zero = true;  // the second step reads x_0 = 0 as a NULL x_old (nothing to clear)
  } else {
    // ns swaps follow the first step
    if ((ns & 1) == 0) {
      cur = x;
      oth = tmp;
    } else {
      TRY(vec_copy(pr, x, tmp, n, s));
      cur = tmp;
      oth = x;
    }
    TRY(launch_operator(L, OP_CHEB, cur, oth, b, cur, 0.0, th[0], nullptr, s));
    std::swap(cur, oth);
  }
  for (int j = 1; j < ns; ++j) {
    TRY(launch_operator(L, OP_CHEB, cur, oth, b, j == 1 && x0_zero ? nullptr : oth, sig[j], th[j], nullptr, s));
    std::swap(cur, oth);
  }
  if (cur != x) return fail(HMG_ERR_INVALID, "internal: Chebyshev buffer parity");
  return HMG_OK;
}

extern "C" int hmg_chebyshev_smooth(const hmg_level* L, const void* b, void* x, int degree,
                                    double lmax, double lof, double hif, int x_is_zero,
                                    hipStream_t s) {
  TRY(check_level(L));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(x, "x"));
  if (degree < 1 || !(lmax > 0) || !(hif > lof) || !(lof > 0))
    return fail(HMG_ERR_INVALID, "need degree >= 1, lmax > 0, 0 < lo_frac < hi_frac");
  return chebyshev(L, b, x, degree, lmax, lof, hif, x_is_zero, s);
}

extern "C" int hmg_rhs_sine(const hmg_level* L, double freq, void* b, hipStream_t s) {
  TRY(check_level(L));
  TRY(check_ptr(b, "b"));
  if (L->space != HMG_DG) return fail(HMG_ERR_UNSUPPORTED, "rhs only for DG levels");
  std::vector<double> h;
  TRY(rhs_sine_host(L->mesh, L->basis, L->geom, freq, h));
  std::vector<char> keep;
  if (L->prec == HMG_F64) return upload<double>(h, b, s, keep);
  return upload<float>(h, b, s, keep);
}

// ================================================================== transfers
struct hmg_transfer {
  const hmg_level* f = nullptr;
  const hmg_level* c = nullptr;
  char kind = 'p';
  std::vector<double> P0, P1;
  size_t ws_bytes = 0, off_sf = 0, off_sc = 0;
  char* ws = nullptr;
  bool fe = false;
};

static bool same_box(const Mesh& a, const Mesh& b) {
  for (int d = 0; d < 3; ++d)
    if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
  for (int f = 0; f < 6; ++f)
    if (a.bc[f] != b.bc[f]) return false;
  return a.curved == b.curved && a.amp == b.amp && a.waves == b.waves && a.mapdeg == b.mapdeg;
}

extern "C" int hmg_transfer_create(const hmg_level* fine, const hmg_level* coarse, char kind,
                                   hmg_transfer** out) {
  if (!fine || !coarse || !out) return fail(HMG_ERR_INVALID, "NULL argument");
  if (fine->prec != coarse->prec) return fail(HMG_ERR_INVALID, "levels differ in precision");
  if (!same_box(fine->mesh, coarse->mesh)) return fail(HMG_ERR_INVALID, "levels differ in domain");
  auto* T = new hmg_transfer();
  T->f = fine;
  T->c = coarse;
  T->kind = kind;
  const Mesh &mf = fine->mesh, &mc = coarse->mesh;
  bool ok = false;
  if (kind == 'c') {
    ok = fine->space == HMG_DG && coarse->space == HMG_FE && fine->k == coarse->k;
    for (int d = 0; d < 3; ++d) ok = ok && mf.N[d] == mc.N[d];
  } else if (kind == 'p') {
    ok = fine->space == coarse->space && coarse->k < fine->k;
    for (int d = 0; d < 3; ++d) ok = ok && mf.N[d] == mc.N[d];
    if (ok) lagrange(coarse->basis.gll, fine->basis.gll, &T->P0, nullptr);
  } else if (kind == 'h') {
    ok = fine->space == coarse->space && coarse->k == fine->k;
    for (int d = 0; d < 3; ++d) ok = ok && mf.N[d] == 2 * mc.N[d];
    if (ok) {
      std::vector<double> x0(fine->n), x1(fine->n);
      for (int i = 0; i < fine->n; ++i) {
        x0[i] = 0.5 * fine->basis.gll[i];
        x1[i] = 0.5 * (1.0 + fine->basis.gll[i]);
      }
      lagrange(coarse->basis.gll, x0, &T->P0, nullptr);
      lagrange(coarse->basis.gll, x1, &T->P1, nullptr);
    }
  }
  if (!ok) {
    delete T;
    return fail(HMG_ERR_INVALID, std::string("levels do not form a '") + kind + "' transfer");
  }
  T->fe = kind != 'c' && fine->space == HMG_FE;
  const size_t es = fine->elem_size();
  if (T->fe) {
    T->off_sf = 0;
    T->off_sc = align256((size_t)fine->n_dg * es);
    T->ws_bytes = T->off_sc + align256((size_t)coarse->n_dg * es);
  }
  *out = T;
  return HMG_OK;
}

extern "C" int hmg_transfer_query(const hmg_transfer* T, size_t* ws) {
  if (!T) return fail(HMG_ERR_INVALID, "transfer is NULL");
  if (ws) *ws = T->ws_bytes;
  return HMG_OK;
}
extern "C" int hmg_transfer_bind(hmg_transfer* T, void* ws, size_t bytes) {
  if (!T) return fail(HMG_ERR_INVALID, "transfer is NULL");
  if (T->ws_bytes == 0) return HMG_OK;
  if (!ws || (((uintptr_t)ws) & 255) || bytes < T->ws_bytes)
    return fail(HMG_ERR_WORKSPACE, "transfer workspace missing, misaligned or too small");
  T->ws = (char*)ws;
  return HMG_OK;
}
extern "C" void hmg_transfer_destroy(hmg_transfer* T) { delete T; }

static int transfer_ready(const hmg_transfer* T) {
  if (!T) return fail(HMG_ERR_INVALID, "transfer is NULL");
  if (T->fe && !T->ws) return fail(HMG_ERR_WORKSPACE, "transfer is not bound");
  return HMG_OK;
}

static int prolongate_add(const hmg_transfer* T, const void* coarse, void* fine, hipStream_t s) {
  const hmg_level *F = T->f, *C = T->c;
  const int pr = F->prec;
  if (T->kind == 'c') return tr_c_inject(pr, F->mesh, F->k, coarse, fine, 0, 1, s);
  const int kind = T->kind == 'h' ? 1 : 0;
  const double* P1 = T->P1.empty() ? nullptr : T->P1.data();
  if (!T->fe)
    return tr_dg_prolongate(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, coarse, fine, 1, s);
  void* sf = T->ws + T->off_sf;
  void* sc = T->ws + T->off_sc;
  TRY(tr_c_inject(pr, C->mesh, C->k, coarse, sc, 0, 0, s));
  TRY(tr_dg_prolongate(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, sc, sf, 0, s));
  return tr_c_sum(pr, F->mesh, F->k, sf, fine, 1, 1, s);
}

static int restrict_(const hmg_transfer* T, const void* fine, void* coarse, hipStream_t s) {
  const hmg_level *F = T->f, *C = T->c;
  const int pr = F->prec;
  if (T->kind == 'c') return tr_c_sum(pr, F->mesh, F->k, fine, coarse, 0, 0, s);
  const int kind = T->kind == 'h' ? 1 : 0;
  const double* P1 = T->P1.empty() ? nullptr : T->P1.data();
  if (!T->fe)
    return tr_dg_restrict(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, fine, coarse, s);
  void* sf = T->ws + T->off_sf;
  void* sc = T->ws + T->off_sc;
  TRY(tr_c_inject(pr, F->mesh, F->k, fine, sf, 1, 0, s));
  TRY(tr_dg_restrict(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, sf, sc, s));
  return tr_c_sum(pr, C->mesh, C->k, sc, coarse, 0, 0, s);
}

extern "C" int hmg_prolongate_add(const hmg_transfer* T, const void* coarse, void* fine, hipStream_t s) {
  TRY(transfer_ready(T));
  TRY(check_ptr(coarse, "coarse"));
  TRY(check_ptr(fine, "fine"));
  return prolongate_add(T, coarse, fine, s);
}
extern "C" int hmg_restrict(const hmg_transfer* T, const void* fine, void* coarse, hipStream_t s) {
  TRY(transfer_ready(T));
  TRY(check_ptr(coarse, "coarse"));
  TRY(check_ptr(fine, "fine"));
  return restrict_(T, fine, coarse, s);
}

// ================================================================== hierarchy
struct hmg_hierarchy {
  Mesh mesh;
  int pseq = 1, h_min = 4, ns = 5, mg_prec = HMG_F64;
  uint64_t seed = 1;
  std::vector<hmg_level*> lv;       // V-cycle levels, fine -> coarse, in mg_prec
  std::vector<hmg_transfer*> tr;    // tr[l]: lv[l] <-> lv[l+1]
  std::vector<double> lmax;
  hmg_level* fine64 = nullptr;      // outer-CG operator (== lv[0] when mg_prec is F64)
  hmg_level* coarse64 = nullptr;    // FP64 copy of the coarsest level (probing)
  bool own_fine64 = false, own_coarse64 = false;
  int64_t nc = 0;                   // coarse unknowns
  // workspace layout
  size_t ws_bytes = 0;
  std::vector<size_t> off_lv, off_tr, off_b, off_x, off_r;
  size_t off_f64 = 0, off_c64 = 0, off_ainv = 0, off_cg = 0, off_part = 0, off_scal = 0, off_c64v = 0;
  // several right-hand sides solved together (hmg_pcg_solve_batched): per
  // level blocks of max_rhs vectors (b, x, r, Chebyshev temporary) ld[l]
  // values apart, and FP64 CG blocks (b, x, r, p, v, z) ld64 values apart
  int max_rhs = 1;
  std::vector<int64_t> ldl;
  std::vector<size_t> off_bb, off_xb, off_rb, off_tb, off_sb;  // off_sb: FE element-local results
  int64_t ld64 = 0;
  size_t off_cgb = 0, off_partb = 0, off_scalb = 0, off_actb = 0, off_dotb = 0;
  char* ws = nullptr;
  bool bound = false;
  // launch graphs (hmg_hierarchy_set_graph): one PCG iteration and one
  // V-cycle, recorded on a library stream, keyed by the caller's vectors
  bool use_graph = false;
  // coarsest-level solve: exact (dense inverse), Chebyshev smoothing only, or
  // the learned correction accepted by its coarse residual (exact fallback)
  int coarse_mode = HMG_COARSE_EXACT;
  hmg_net* net = nullptr;
  double accept = 0.0;
  double c0 = 1.0;   // output scale of the network: 1 / mean free diagonal of the coarse operator
  double lmax_c = 0.0;
  bool dense = true;          // dense inverse of the coarsest operator (<= 8192 unknowns)
  double coarse_rtol = 1e-3;  // iterative coarse solve: Jacobi-PCG tolerance and iteration cap
  int coarse_maxit = 50;
  bool flexible = false;
  int64_t net_version = -1;  // network parameters the recorded graphs saw
  // coarse right-hand sides of eager V-cycles copied to a caller buffer (FP64)
  double* cap_buf = nullptr;
  int cap_capacity = 0, cap_count = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t it_exec = nullptr, vc_exec = nullptr;
  const void *it_x = nullptr, *vc_b = nullptr, *vc_x = nullptr;
  void drop_graphs() {
    if (it_exec) (void)hipGraphExecDestroy(it_exec);
    if (vc_exec) (void)hipGraphExecDestroy(vc_exec);
    it_exec = vc_exec = nullptr;
    it_x = vc_b = vc_x = nullptr;
  }
  void* b(int l) const { return ws + off_b[l]; }
  void* x(int l) const { return ws + off_x[l]; }
  void* r(int l) const { return ws + off_r[l]; }
  double* cg(int i) const { return (double*)(ws + off_cg) + (size_t)i * fine64->n_dofs; }
  double* part() const { return (double*)(ws + off_part); }
  double* scal() const { return (double*)(ws + off_scal); }
  double* ainv() const { return (double*)(ws + off_ainv); }
  void* bb(int l) const { return ws + off_bb[l]; }
  void* xb(int l) const { return ws + off_xb[l]; }
  void* rb(int l) const { return ws + off_rb[l]; }
  void* tb(int l) const { return ws + off_tb[l]; }
  void* sb(int l) const { return lv[l]->space == HMG_FE ? (void*)(ws + off_sb[l]) : nullptr; }
  double* cgb(int i) const { return (double*)(ws + off_cgb) + (size_t)i * max_rhs * ld64; }
  double* partb() const { return (double*)(ws + off_partb); }
  double* scalb(int i) const { return (double*)(ws + off_scalb) + (size_t)i * max_rhs; }  // 0..5
  int* actb() const { return (int*)(ws + off_actb); }
  // per-item partials of p.(A p) from the several-vector FP64 apply (degree 6
  // and 7), n_el * max_rhs values; NULL where the apply cannot write them
  double* dotb() const { return fine64->n >= 7 ? (double*)(ws + off_dotb) : nullptr; }
  // FP64 right-hand side and solution of the iterative coarse solve when the
  // V-cycle runs in FP32 (the coarse solve itself is an FP64 step)
  double* cb64() const { return (double*)(ws + off_c64v); }
  double* cx64() const { return (double*)(ws + off_c64v) + nc; }
  ~hmg_hierarchy() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
    for (auto* t : tr) delete t;
    if (own_fine64) delete fine64;
    if (own_coarse64) delete coarse64;
    for (auto* l : lv) delete l;
  }
};

static void hierarchy_layout(hmg_hierarchy* H);

static bool can_h(const Mesh& m, int h_min) {
  for (int d = 0; d < 3; ++d)
    if (m.N[d] % 2) return false;
  return std::max(m.N[0], std::max(m.N[1], m.N[2])) > h_min;
}

extern "C" int hmg_hierarchy_create(const hmg_mesh_desc* desc, const char* strategy, int pseq,
                                    int h_min, int ns, int mg_prec, uint64_t seed,
                                    hmg_hierarchy** out) {
  if (!out || !strategy) return fail(HMG_ERR_INVALID, "NULL argument");
  if (pseq < 0 || pseq > 2 || ns < 1 || (mg_prec != HMG_F64 && mg_prec != HMG_F32))
    return fail(HMG_ERR_INVALID, "bad pseq, smoother degree or precision");
  for (const char* c = strategy; *c; ++c)
    if (*c != 'c' && *c != 'p' && *c != 'h') return fail(HMG_ERR_INVALID, "strategy letters are c, p, h");
  Mesh m;
  TRY(to_mesh(desc, m));
  auto* H = new hmg_hierarchy();
  H->mesh = m;
  H->pseq = pseq;
  H->h_min = h_min < 1 ? 1 : h_min;
  H->ns = ns;
  H->mg_prec = mg_prec;
  H->seed = seed;
  // level specs (Sec. 3.2: one of h, p, c changes per level)
  struct Spec { int space; Mesh m; char kind; };
  std::vector<Spec> specs{{HMG_DG, m, 0}};
  for (const char* c = strategy; *c; ++c) {
    Spec cur = specs.back();
    if (*c == 'c' && cur.space == HMG_DG) {
      specs.back().kind = 'c';
      specs.push_back({HMG_FE, cur.m, 0});
    } else if (*c == 'p') {
      while (specs.back().m.k > 1) {
        Spec nx = specs.back();
        int k = nx.m.k;
        nx.m.k = pseq == 0 ? k - 1 : (pseq == 1 ? k / 2 : 1);
        specs.back().kind = 'p';
        nx.kind = 0;
        specs.push_back(nx);
      }
    } else if (*c == 'h') {
      while (can_h(specs.back().m, H->h_min)) {
        Spec nx = specs.back();
        for (int d = 0; d < 3; ++d) nx.m.N[d] /= 2;
        if (!nx.m.tau_scale.empty()) {  // parent penalty scale: mean of the children
          std::vector<double> ts((size_t)nx.m.n_el(), 0.0);
          const Mesh& fm = specs.back().m;
          for (int64_t e = 0; e < fm.n_el(); ++e) {
            int64_t ex = e % fm.N[0], ey = (e / fm.N[0]) % fm.N[1], ez = e / ((int64_t)fm.N[0] * fm.N[1]);
            ts[(ex / 2) + nx.m.N[0] * ((ey / 2) + (int64_t)nx.m.N[1] * (ez / 2))] += fm.tau_scale[e] / 8.0;
          }
          nx.m.tau_scale = ts;
        }
        specs.back().kind = 'h';
        nx.kind = 0;
        specs.push_back(nx);
      }
    }
  }
  for (auto& sp : specs) {
    hmg_level* L = nullptr;
    int rc = level_init(sp.m, sp.space, mg_prec, &L);
    if (rc) {
      delete H;
      return rc;
    }
    H->lv.push_back(L);
  }
  for (size_t l = 0; l + 1 < specs.size(); ++l) {
    hmg_transfer* T = nullptr;
    int rc = hmg_transfer_create(H->lv[l], H->lv[l + 1], specs[l].kind, &T);
    if (rc) {
      delete H;
      return rc;
    }
    H->tr.push_back(T);
  }
  H->lmax.assign(H->lv.size(), 0.0);
  if (mg_prec == HMG_F64) {
    H->fine64 = H->lv[0];
    H->coarse64 = H->lv.back();
  } else {
    int rc = level_init(m, HMG_DG, HMG_F64, &H->fine64);
    if (!rc) rc = level_init(specs.back().m, specs.back().space, HMG_F64, &H->coarse64);
    H->own_fine64 = H->own_coarse64 = true;
    if (rc) {
      delete H;
      return rc;
    }
  }
  H->nc = H->lv.back()->n_dofs;
  // dense inverse up to 8192 unknowns; above, the coarse solve is iterative
  H->dense = H->nc <= 8192;
  H->coarse_mode = H->dense ? HMG_COARSE_EXACT : HMG_COARSE_CG;
  hierarchy_layout(H);
  *out = H;
  return HMG_OK;
}

// Values between consecutive vectors of a block: n rounded up to 256 bytes.
static int64_t block_ld(int64_t n, size_t es) {
  const int64_t per = 256 / (int64_t)es;
  return (n + per - 1) / per * per;
}

// Workspace layout of a hierarchy (byte offsets and total size).
static void hierarchy_layout(hmg_hierarchy* H) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  H->off_lv.clear();
  H->off_tr.clear();
  H->off_b.clear();
  H->off_x.clear();
  H->off_r.clear();
  H->off_bb.clear();
  H->off_xb.clear();
  H->off_rb.clear();
  H->off_tb.clear();
  H->off_sb.clear();
  H->ldl.clear();
  for (auto* L : H->lv) H->off_lv.push_back(take(L->ws_bytes));
  for (auto* T : H->tr) H->off_tr.push_back(take(T->ws_bytes));
  for (auto* L : H->lv) {
    H->off_b.push_back(take(L->vec_bytes()));
    H->off_x.push_back(take(L->vec_bytes()));
    H->off_r.push_back(take(L->vec_bytes()));
  }
  if (H->own_fine64) {
    H->off_f64 = take(H->fine64->ws_bytes);
    H->off_c64 = take(H->coarse64->ws_bytes);
  }
  H->off_ainv = take(H->dense ? (size_t)H->nc * H->nc * 8 : 8);
  H->off_c64v = take(H->own_coarse64 ? (size_t)2 * H->nc * 8 : 8);
  H->off_cg = take((size_t)4 * H->fine64->n_dofs * 8);
  H->off_part = take((size_t)kPartials * 8);
  H->off_scal = take(32 * 8);
  if (H->max_rhs > 1) {
    const size_t m = (size_t)H->max_rhs;
    for (auto* L : H->lv) {
      const int64_t ld = block_ld(L->n_dofs, L->elem_size());
      H->ldl.push_back(ld);
      H->off_bb.push_back(take(m * ld * L->elem_size()));
      H->off_xb.push_back(take(m * ld * L->elem_size()));
      H->off_rb.push_back(take(m * ld * L->elem_size()));
      H->off_tb.push_back(take(m * ld * L->elem_size()));
      H->off_sb.push_back(take(L->space == HMG_FE ? m * L->n_dg * L->elem_size() : 0));
    }
    H->ld64 = block_ld(H->fine64->n_dofs, 8);
    H->off_cgb = take(6 * m * H->ld64 * 8);
    H->off_partb = take(m * kPartialsB * 8);
    H->off_scalb = take(6 * m * 8);
    H->off_actb = take(m * sizeof(int));
    H->off_dotb = take(H->fine64->n >= 7 ? m * (size_t)H->fine64->n_el * 8 : 0);
  }
  H->ws_bytes = off;
}

extern "C" int hmg_hierarchy_query(const hmg_hierarchy* H, int64_t* n, size_t* ws) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (n) *n = H->fine64->n_dofs;
  if (ws) *ws = H->ws_bytes;
  return HMG_OK;
}

// Probe the coarsest FP64 operator with coloured unit vectors, assemble the
// dense matrix on the host, factor it and upload its inverse.
static int coarse_setup(hmg_hierarchy* H, hipStream_t s) {
  const hmg_level* C = H->coarse64;
  const int64_t n = C->n_dofs;
  const Mesh& m = C->mesh;
  const int k = C->k, np = k + 1, n3 = np * np * np;
  std::vector<double> A((size_t)n * n, 0.0), e(n), y(n);
  void* du = C->tmp(1);
  void* dv = C->tmp(2);
  const bool fe = C->space == HMG_FE;
  const int Mx = m.N[0] * k + 1, My = m.N[1] * k + 1, Mz = m.N[2] * k + 1;
  const int per = fe ? 2 * k + 1 : 3;
  const int ncol = fe ? per * per * per : 27 * n3;
  for (int c = 0; c < ncol; ++c) {
    std::fill(e.begin(), e.end(), 0.0);
    std::vector<int64_t> cols;
    if (fe) {
      const int cx = c % per, cy = (c / per) % per, cz = c / (per * per);
      for (int gz = cz; gz < Mz; gz += per)
        for (int gy = cy; gy < My; gy += per)
          for (int gx = cx; gx < Mx; gx += per) cols.push_back(gx + (int64_t)Mx * (gy + (int64_t)My * gz));
    } else {
      const int col = c / n3, loc = c % n3;
      const int cx = col % 3, cy = (col / 3) % 3, cz = col / 9;
      for (int ez = cz; ez < m.N[2]; ez += 3)
        for (int ey = cy; ey < m.N[1]; ey += 3)
          for (int ex = cx; ex < m.N[0]; ex += 3)
            cols.push_back((ex + (int64_t)m.N[0] * (ey + (int64_t)m.N[1] * ez)) * n3 + loc);
    }
    if (cols.empty()) continue;
    for (auto j : cols) e[j] = 1.0;
    HMG_HIP(hipMemcpyAsync(du, e.data(), n * 8, hipMemcpyHostToDevice, s));
    TRY(launch_operator(C, OP_APPLY, du, dv, nullptr, nullptr, 0, 0, nullptr, s));
    HMG_HIP(hipMemcpyAsync(y.data(), dv, n * 8, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    // each row sees at most one probed column: attribute it
    for (auto j : cols) {
      if (fe) {
        const int gx = (int)(j % Mx), gy = (int)((j / Mx) % My), gz = (int)(j / ((int64_t)Mx * My));
        for (int z = std::max(0, gz - k); z <= std::min(Mz - 1, gz + k); ++z)
          for (int yy = std::max(0, gy - k); yy <= std::min(My - 1, gy + k); ++yy)
            for (int x = std::max(0, gx - k); x <= std::min(Mx - 1, gx + k); ++x) {
              const int64_t i = x + (int64_t)Mx * (yy + (int64_t)My * z);
              A[(size_t)i * n + j] = y[i];
            }
      } else {
        const int64_t el = j / n3;
        const int ex = (int)(el % m.N[0]), ey = (int)((el / m.N[0]) % m.N[1]),
                  ez = (int)(el / ((int64_t)m.N[0] * m.N[1]));
        const int nb[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
        for (auto& o : nb) {
          const int x = ex + o[0], yy = ey + o[1], z = ez + o[2];
          if (x < 0 || yy < 0 || z < 0 || x >= m.N[0] || yy >= m.N[1] || z >= m.N[2]) continue;
          const int64_t ei = x + (int64_t)m.N[0] * (yy + (int64_t)m.N[1] * z);
          for (int r = 0; r < n3; ++r) A[(size_t)(ei * n3 + r) * n + j] = y[ei * n3 + r];
        }
      }
    }
  }
  // symmetrize (round-off) and factor
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
      A[(size_t)i * n + j] = A[(size_t)j * n + i] = v;
    }
  if (!cholesky(A, (int)n)) return fail(HMG_ERR_BREAKDOWN, "coarse matrix is not positive definite");
  std::vector<double> Ainv;
  chol_inverse(A, (int)n, Ainv);
  HMG_HIP(hipMemcpyAsync(H->ainv(), Ainv.data(), (size_t)n * n * 8, hipMemcpyHostToDevice, s));
  HMG_HIP(hipStreamSynchronize(s));
  return HMG_OK;
}

static NodeGrid coarse_nodes(const hmg_hierarchy* H);

extern "C" int hmg_hierarchy_bind(hmg_hierarchy* H, void* ws, size_t bytes, hipStream_t s) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (!ws || (((uintptr_t)ws) & 255)) return fail(HMG_ERR_WORKSPACE, "workspace NULL or misaligned");
  if (bytes < H->ws_bytes) return fail(HMG_ERR_WORKSPACE, "workspace too small");
  H->drop_graphs();  // recorded launches point into the previous workspace
  H->ws = (char*)ws;
  for (size_t l = 0; l < H->lv.size(); ++l)
    TRY(hmg_level_bind(H->lv[l], H->ws + H->off_lv[l], H->lv[l]->ws_bytes, s));
  for (size_t l = 0; l < H->tr.size(); ++l)
    TRY(hmg_transfer_bind(H->tr[l], H->ws + H->off_tr[l], H->tr[l]->ws_bytes));
  if (H->own_fine64) {
    TRY(hmg_level_bind(H->fine64, H->ws + H->off_f64, H->fine64->ws_bytes, s));
    TRY(hmg_level_bind(H->coarse64, H->ws + H->off_c64, H->coarse64->ws_bytes, s));
  }
  for (size_t l = 0; l + 1 < H->lv.size(); ++l)
    TRY(estimate_lmax(H->lv[l], 20, H->seed + l, &H->lmax[l], s));
  TRY(estimate_lmax(H->lv.back(), 20, H->seed + H->lv.size(), &H->lmax_c, s));
  if (H->dense) TRY(coarse_setup(H, s));
  {  // network output scale: 1 / mean diagonal over the free coarse unknowns
    const hmg_level* C = H->coarse64;
    const NodeGrid ng = coarse_nodes(H);
    double sd = 0;
    int64_t nd = 0;
    for (int64_t i = 0; i < (int64_t)C->diag_h.size(); ++i) {
      bool fixed = false;
      if (C->space == HMG_FE) {
        const int x = (int)(i % ng.Mx), y = (int)((i / ng.Mx) % ng.My), z = (int)(i / ((int64_t)ng.Mx * ng.My));
        const int m = ng.bcmask;
        fixed = (x == 0 && !(m & 1)) || (x == ng.Mx - 1 && !(m & 2)) || (y == 0 && !(m & 4)) ||
                (y == ng.My - 1 && !(m & 8)) || (z == 0 && !(m & 16)) || (z == ng.Mz - 1 && !(m & 32));
      }
      if (!fixed) {
        sd += C->diag_h[i];
        ++nd;
      }
    }
    H->c0 = nd > 0 && sd > 0 ? nd / sd : 1.0;
  }
  {
    std::vector<double> zero(32, 0.0);
    HMG_HIP(hipMemcpyAsync(H->scal(), zero.data(), 32 * 8, hipMemcpyHostToDevice, s));
    HMG_HIP(hipStreamSynchronize(s));
  }
  H->bound = true;
  return HMG_OK;
}

extern "C" void hmg_hierarchy_destroy(hmg_hierarchy* H) { delete H; }

extern "C" int hmg_hierarchy_levels(const hmg_hierarchy* H, int* n) {
  if (!H || !n) return fail(HMG_ERR_INVALID, "NULL argument");
  *n = (int)H->lv.size();
  return HMG_OK;
}
extern "C" int hmg_hierarchy_level_info(const hmg_hierarchy* H, int l, hmg_level_info* info) {
  if (!H || !info) return fail(HMG_ERR_INVALID, "NULL argument");
  if (l < 0 || l >= (int)H->lv.size()) return fail(HMG_ERR_INVALID, "level index out of range");
  const hmg_level* L = H->lv[l];
  info->space = L->space;
  info->degree = L->k;
  for (int d = 0; d < 3; ++d) info->nel[d] = L->mesh.N[d];
  info->prec = L->prec;
  info->n_dofs = L->n_dofs;
  info->lmax = H->lmax[l];
  return HMG_OK;
}
extern "C" int hmg_hierarchy_set_lmax(hmg_hierarchy* H, int l, double lmax) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (l < 0 || l + 1 >= (int)H->lv.size() || !(lmax > 0)) return fail(HMG_ERR_INVALID, "bad level or lmax");
  H->lmax[l] = lmax;
  return HMG_OK;
}

// Alg. 2 on level l with x^(l) = 0; b(l) holds the right-hand side.
static NodeGrid coarse_nodes(const hmg_hierarchy* H) {
  const hmg_level* C = H->lv.back();
  NodeGrid ng;
  ng.Mx = C->mesh.N[0] * C->k + 1;
  ng.My = C->mesh.N[1] * C->k + 1;
  ng.Mz = C->mesh.N[2] * C->k + 1;
  ng.bcmask = C->mesh.bcmask();
  return ng;
}

// Jacobi-preconditioned CG (Alg. 1 with D^{-1}) for L x = b, x_0 = 0, at most
// maxit iterations, stopping on the GPU once r.z <= rtol^2 r_0.z_0: every
// later kernel returns at once (the gate *skip), so the sequence can be
// recorded.  Eager launches also read the gate every 8 iterations and stop
// early.  *skip must be set before the call (nonzero: do nothing).
// Scalars: sc[16..17] r.z (alternating), sc[18] p.q, sc[19] r_0.z_0.
static int coarse_cg(hmg_hierarchy* H, const hmg_level* L, const void* b, void* x, double rtol, int maxit,
                     hipStream_t s) {
  const int pr = L->prec;
  const int64_t n = L->n_dofs;
  void *r = L->tmp(0), *z = L->tmp(1), *p = L->tmp(2), *q = L->tmp(3);
  double* sc = H->scal() + 16;
  int* skip = (int*)(H->scal() + 24);
  int* iters = skip + 1;
  double* part = H->part();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HMG_HIP(hipStreamIsCapturing(s, &cs));
  const bool eager = cs == hipStreamCaptureStatusNone;
  if (eager) {  // a solve the gate already skips costs no launches
    int done = 0;
    HMG_HIP(hipMemcpyAsync(&done, skip, sizeof(int), hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    if (done) return HMG_OK;
  }
  TRY(ccg_init(pr, b, L->dinv(), x, r, z, p, n, skip, s));
  TRY(vec_dot_gated(pr, r, z, n, part, sc + 0, skip, s));
  TRY(vec_dot_gated(pr, r, z, n, part, sc + 3, skip, s));
  for (int it = 0; it < maxit; ++it) {
    double* old = sc + (it & 1);
    double* nw = sc + ((it + 1) & 1);
    TRY(launch_operator_gated(L, OP_APPLY, p, q, nullptr, skip, s));
    TRY(vec_dot_gated(pr, p, q, n, part, sc + 2, skip, s));
    TRY(ccg_xr(pr, x, r, z, p, q, L->dinv(), n, old, sc + 2, skip, s));
    TRY(vec_dot_gated(pr, r, z, n, part, nw, skip, s));
    TRY(ccg_p(pr, p, z, n, nw, old, skip, s));
    TRY(ccg_check(nw, sc + 3, rtol * rtol, skip, iters, s));
    if (eager && (it & 7) == 7) {
      int done = 0;
      HMG_HIP(hipMemcpyAsync(&done, skip, sizeof(int), hipMemcpyDeviceToHost, s));
      HMG_HIP(hipStreamSynchronize(s));
      if (done) break;
    }
  }
  return HMG_OK;
}

// The iterative coarse solve, always in FP64: on the FP64 copy of the
// coarsest level, the level-precision right-hand side converted on the way
// in and the solution converted back.  *skip (set before the call) gates
// the conversion in and the solve.  The solve sets *skip once it has
// converged, so the conversion back is gated by the acceptance test
// *accepted instead (0 outside the learned correction).
static int coarse_cg64_at(hmg_hierarchy* H, size_t l, const void* b, void* x, hipStream_t s) {
  hmg_level* L = H->lv[l];
  if (!H->own_coarse64) return coarse_cg(H, L, b, x, H->coarse_rtol, H->coarse_maxit, s);
  int* skip = (int*)(H->scal() + 24);
  int* accepted = skip + 2;
  TRY(vec_convert_gated(L->prec, b, HMG_F64, H->cb64(), H->nc, skip, s));
  TRY(coarse_cg(H, H->coarse64, H->cb64(), H->cx64(), H->coarse_rtol, H->coarse_maxit, s));
  return vec_convert_gated(HMG_F64, H->cx64(), L->prec, x, H->nc, accepted, s);
}
static int coarse_cg64(hmg_hierarchy* H, size_t l, hipStream_t s) { return coarse_cg64_at(H, l, H->b(l), H->x(l), s); }

// Coarsest level: x(l) from b(l) by the selected coarse solve.
static int coarse_solve(hmg_hierarchy* H, size_t l, hipStream_t s) {
  hmg_level* L = H->lv[l];
  if (H->cap_buf && H->cap_count < H->cap_capacity) {
    TRY(vec_convert(L->prec, H->b(l), HMG_F64, H->cap_buf + (size_t)H->cap_count * H->nc, H->nc, s));
    H->cap_count++;
  }
  int* skip = (int*)(H->scal() + 24);
  switch (H->coarse_mode) {
    case HMG_COARSE_SMOOTH:
      return chebyshev(L, H->b(l), H->x(l), H->ns, H->lmax_c, 0.06, 1.2, 1, s);
    case HMG_COARSE_CG:
      TRY(set_flag(skip, 0, s));
      if (H->own_coarse64) TRY(set_flag(skip + 2, 0, s));
      return coarse_cg64(H, l, s);
    case HMG_COARSE_LEARNED: {
      hmg_net* N = H->net;
      const NodeGrid ng = coarse_nodes(H);
      TRY(net_pack(L->prec, H->b(l), nullptr, H->nc, 1, ng, N->G, H->c0, net_hsigma(N), net_hin(N), nullptr, s));
      TRY(net_forward(N, net_hin(N), net_hout(N), 1, s));
      TRY(net_unpack(L->prec, net_hout(N), ng, N->G, net_hsigma(N), H->c0, H->x(l), s));
      // acceptance test: |b - A x| against accept |b|, else the exact solve
      double* gate = H->scal() + 8;
      TRY(launch_operator(L, OP_RESID, H->x(l), H->r(l), H->b(l), nullptr, 0, 0, nullptr, s));
      TRY(vec_dot(L->prec, H->r(l), H->r(l), H->nc, H->part(), gate, s));
      TRY(vec_dot(L->prec, H->b(l), H->b(l), H->nc, H->part(), gate + 1, s));
      if (H->dense)
        return coarse_gemv_gated(L->prec, H->ainv(), H->b(l), H->x(l), (int)H->nc, gate, H->accept,
                                 (int*)(H->scal() + 10), s);
      // no dense inverse: the iterative coarse solve runs only for a rejected correction
      TRY(gate_to_skip(gate, H->accept, skip, (int*)(H->scal() + 10), s, skip + 2));
      return coarse_cg64(H, l, s);
    }
    default:
      return coarse_gemv(L->prec, H->ainv(), H->b(l), H->x(l), (int)H->nc, s);
  }
}

static int vcycle(hmg_hierarchy* H, size_t l, hipStream_t s) {
  hmg_level* L = H->lv[l];
  if (l + 1 == H->lv.size()) return coarse_solve(H, l, s);
  TRY(chebyshev(L, H->b(l), H->x(l), H->ns, H->lmax[l], 0.06, 1.2, 1, s));
  TRY(launch_operator(L, OP_RESID, H->x(l), H->r(l), H->b(l), nullptr, 0, 0, nullptr, s));
  TRY(restrict_(H->tr[l], H->r(l), H->b(l + 1), s));
  TRY(vcycle(H, l + 1, s));
  TRY(prolongate_add(H->tr[l], H->x(l + 1), H->x(l), s));
  return chebyshev(L, H->b(l), H->x(l), H->ns, H->lmax[l], 0.06, 1.2, 0, s);
}

// Record body(stream) once as a HIP graph on the hierarchy's own stream
// (default priority; nothing is executed while recording) and instantiate it.
template <class Body>
static int record(hmg_hierarchy* H, hipGraphExec_t* exec, Body&& body) {
  if (!H->cap) HMG_HIP(hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking));
  if (*exec) {
    (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  HMG_HIP(hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal));
  const int rc = body(H->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(H->cap, &g);
  if (rc != HMG_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != HMG_OK ? rc : fail(HMG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    *exec = nullptr;
    return fail(HMG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  return HMG_OK;
}

extern "C" int hmg_hierarchy_set_graph(hmg_hierarchy* H, int enable) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  H->use_graph = enable != 0;
  if (!H->use_graph) H->drop_graphs();
  return HMG_OK;
}

// Before a solve or V-cycle with the learned coarse solve: BF16 weights up
// to date (outside any recording) and recordings made with older
// parameters dropped.
static int learned_ready(hmg_hierarchy* H, hipStream_t s) {
  if (H->coarse_mode != HMG_COARSE_LEARNED) return HMG_OK;
  TRY(net_prepare(H->net, s));
  if (H->net->version != H->net_version) {
    H->drop_graphs();
    H->net_version = H->net->version;
  }
  return HMG_OK;
}

static int precondition(hmg_hierarchy* H, const double* b, double* x, hipStream_t s) {
  const int pr = H->mg_prec;
  const int64_t n = H->lv[0]->n_dofs;
  TRY(vec_convert(HMG_F64, b, pr, H->b(0), n, s));
  TRY(vcycle(H, 0, s));
  return vec_convert(pr, H->x(0), HMG_F64, x, n, s);
}

extern "C" int hmg_vcycle(hmg_hierarchy* H, const double* b, double* x, hipStream_t s) {
  if (!H || !H->bound) return fail(HMG_ERR_WORKSPACE, "hierarchy missing or not bound");
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(x, "x"));
  if ((const void*)b == (void*)x) return fail(HMG_ERR_INVALID, "b and x must not overlap");
  TRY(learned_ready(H, s));
  if (!H->use_graph || H->cap_buf) return precondition(H, b, x, s);
  if (!H->vc_exec || H->vc_b != b || H->vc_x != x) {
    TRY(record(H, &H->vc_exec, [&](hipStream_t cs) { return precondition(H, b, x, cs); }));
    H->vc_b = b;
    H->vc_x = x;
  }
  HMG_HIP(hipGraphLaunch(H->vc_exec, s));
  return HMG_OK;
}

// The second half of a PCG iteration (Alg. 1): v = A p, p.Ap -> sc[2],
// alpha = sc[1] / sc[2], x += alpha p, r -= alpha v, r.r -> sc[3], and the
// current delta kept in sc[0] for the next beta.
// FP32 V-cycle inside standard CG: the CG update also writes r in FP32 into
// the V-cycle's right-hand side, and r.z and the direction update read the
// V-cycle's FP32 result (widened exactly, as a conversion to FP64 would), so
// z is never stored in FP64 (the same arithmetic, three passes fewer).
static bool fp32_z(const hmg_hierarchy* H) { return !H->flexible && H->mg_prec == HMG_F32; }

static int pcg_update(hmg_hierarchy* H, double* x, hipStream_t s) {
  const hmg_level* A = H->fine64;
  const int64_t n = A->n_dofs;
  double *r = H->cg(0), *p = H->cg(1), *v = H->cg(2), *sc = H->scal(), *part = H->part();
  int nparts = 0;
  TRY(launch_operator(A, OP_DOT, p, v, nullptr, nullptr, 0, 0, &nparts, s));
  TRY(reduce_partials(A->partials(), nparts, sc + 2, s));
  const int g = cg_update_xr(x, r, p, v, sc + 1, sc + 2, n, part, s, sc + 0,
                             fp32_z(H) ? (float*)H->b(0) : nullptr);
  if (g < 0) return g;
  return reduce_partials(part, g, sc + 3, s);
}

// A full PCG iteration after the first: z = M^{-1} r (V-cycle), delta =
// r.z -> sc[1], p = z + (sc[1] / sc[0]) p, then pcg_update.
// Flexible variant (a preconditioner that changes between iterations, such
// as the learned coarse correction): beta = z_{k+1}.(r_{k+1} - r_k) /
// (r_k.z_k) = -(z_{k+1}.A p_k) / (p_k.A p_k), with A p_k still in v.
static int pcg_iteration(hmg_hierarchy* H, double* x, hipStream_t s) {
  const int64_t n = H->fine64->n_dofs;
  double *r = H->cg(0), *p = H->cg(1), *v = H->cg(2), *z = H->cg(3), *sc = H->scal(), *part = H->part();
  if (fp32_z(H)) {  // the right-hand side H->b(0) holds r in FP32 (pcg_update)
    TRY(vcycle(H, 0, s));
    const float* z32 = (const float*)H->x(0);
    TRY(vec_dot_zf(r, z32, n, part, sc + 1, s));
    TRY(cg_update_p_zf(p, z32, sc + 1, sc + 0, n, s));
    return pcg_update(H, x, s);
  }
  TRY(precondition(H, r, z, s));
  TRY(vec_dot(HMG_F64, r, z, n, part, sc + 1, s));
  if (H->flexible) {
    TRY(vec_dot(HMG_F64, z, v, n, part, sc + 4, s));
    TRY(cg_update_p(p, z, sc + 4, sc + 2, n, s, true));
  } else {
    TRY(cg_update_p(p, z, sc + 1, sc + 0, n, s));
  }
  return pcg_update(H, x, s);
}

extern "C" int hmg_pcg_solve(hmg_hierarchy* H, const double* b, double* x, double rtol, double atol,
                             int maxit, hmg_solve_stats* st, hipStream_t s) {
  if (!H || !H->bound) return fail(HMG_ERR_WORKSPACE, "hierarchy missing or not bound");
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(x, "x"));
  if (maxit < 0) return fail(HMG_ERR_INVALID, "maxit < 0");
  TRY(learned_ready(H, s));
  const hmg_level* A = H->fine64;
  const int64_t n = A->n_dofs;
  double *r = H->cg(0), *p = H->cg(1), *z = H->cg(3);
  double* sc = H->scal();  // 0: previous delta, 1: delta = r.z, 2: p.Ap, 3: r.r
  double* part = H->part();
  hmg_solve_stats stats{0, 0, 0, 0, 0};
  auto finish = [&](int code) {
    if (st) *st = stats;
    return code;
  };
  TRY(launch_operator(A, OP_RESID, x, r, b, nullptr, 0, 0, nullptr, s));
  TRY(vec_dot(HMG_F64, r, r, n, part, sc + 3, s));
  double rr;
  HMG_HIP(hipMemcpyAsync(&rr, sc + 3, 8, hipMemcpyDeviceToHost, s));
  HMG_HIP(hipStreamSynchronize(s));
  double nr = std::sqrt(rr);
  stats.r0 = stats.rn = nr;
  if (!std::isfinite(nr)) return finish(fail(HMG_ERR_NONFINITE, "initial residual is not finite"));
  const double r0 = nr;
  if (r0 == 0.0 || nr <= atol) return finish(HMG_OK);
  if (fp32_z(H)) {
    TRY(vec_convert(HMG_F64, r, HMG_F32, H->b(0), n, s));
    TRY(vcycle(H, 0, s));
    TRY(cg_update_p_zf(p, (const float*)H->x(0), nullptr, nullptr, n, s));
    TRY(vec_dot_zf(r, (const float*)H->x(0), n, part, sc + 1, s));
  } else {
    TRY(precondition(H, r, z, s));
    TRY(vec_copy(HMG_F64, z, p, n, s));
    TRY(vec_dot(HMG_F64, r, z, n, part, sc + 1, s));
  }
  int it = 0;
  while (nr / r0 > rtol && nr > atol && it < maxit) {
    if (it == 0) {
      TRY(pcg_update(H, x, s));
    } else if (H->use_graph && !H->cap_buf) {
      if (!H->it_exec || H->it_x != x) {
        TRY(record(H, &H->it_exec, [&](hipStream_t cs) { return pcg_iteration(H, x, cs); }));
        H->it_x = x;
      }
      HMG_HIP(hipGraphLaunch(H->it_exec, s));
    } else {
      TRY(pcg_iteration(H, x, s));
    }
    double hs[2];
    HMG_HIP(hipMemcpyAsync(hs, sc + 2, 16, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    ++it;
    nr = std::sqrt(hs[1]);
    stats.iters = it;
    stats.rn = nr;
    if (!(hs[0] > 0)) return finish(fail(HMG_ERR_BREAKDOWN, "p^T A p <= 0: operator not SPD"));
    if (!std::isfinite(nr)) return finish(fail(HMG_ERR_NONFINITE, "residual is not finite"));
  }
  if (it > 0) {
    stats.rho = std::pow(nr / r0, 1.0 / it);
    stats.n10 = -10.0 / std::log10(stats.rho);
  }
  if (nr / r0 > rtol && nr > atol) return finish(HMG_NOT_CONVERGED);
  return finish(HMG_OK);
}

// ================================================================== several right-hand sides
// The V-cycle and PCG on blocks of nrhs vectors: every level applies its
// operator to all vectors in one launch (the element geometry read once per
// element for all of them; the node sums of continuous FE levels follow as
// one launch), and so do the transfers; the coarse solve takes the vectors
// one after another.

// Alg. 3 on nrhs vectors (vector r at r * ld); tmp: a block like x;
// fe: the element-local results block of a continuous FE level.
static int chebyshev_v(const hmg_level* L, int nrhs, int64_t ld, const void* b, void* x, void* tmp, int ns,
                       double lmax, int x_is_zero, void* fe, hipStream_t s, void* tmp2 = nullptr) {
  const size_t es = L->elem_size();
  if (L->space != HMG_DG && !fe) {
    for (int r = 0; r < nrhs; ++r)
      TRY(chebyshev(L, (const char*)b + r * ld * es, (char*)x + r * ld * es, ns, lmax, 0.06, 1.2, x_is_zero, s));
    return HMG_OK;
  }
  std::vector<double> sig, th;
  cheb_coeffs(ns, lmax, 0.06, 1.2, sig, th);
  const int pr = L->prec;
  const int64_t n = L->n_dofs, all = ld * nrhs;
  void *cur, *oth;
  bool x0_zero = false;
  if (!x_is_zero && (ns & 1) && ns >= 3 && tmp2) {
    // odd degree from a nonzero start without copying x (see chebyshev)
    void *prev = x, *at = x;
    for (int j = 0; j < ns; ++j) {
      void* out = j == ns - 1 ? x : (j == ns - 2 ? tmp2 : ((j & 1) ? x : tmp));
      TRY(launch_operator_batched(L, OP_CHEB, nrhs, ld, at, out, b, j == 0 ? at : prev, j == 0 ? 0.0 : sig[j],
                                  th[j], nullptr, s, fe));
      prev = at;
      at = out;
    }
    return HMG_OK;
  }
  if (x_is_zero) {
    if (((ns - 1) & 1) == 0) {
      cur = x;
      oth = tmp;
    } else {
      cur = tmp;
      oth = x;
    }
    TRY(vec_mul3_b(pr, th[0], L->dinv(), b, cur, n, ld, nrhs, s));
    x0_zero = true;  // the second step reads x_0 = 0 as a NULL x_old (nothing to clear)
  } else {
    if ((ns & 1) == 0) {
      cur = x;
      oth = tmp;
    } else {
      TRY(vec_copy(pr, x, tmp, all, s));
      cur = tmp;
      oth = x;
    }
    TRY(launch_operator_batched(L, OP_CHEB, nrhs, ld, cur, oth, b, cur, 0.0, th[0], nullptr, s, fe));
    std::swap(cur, oth);
  }
  for (int j = 1; j < ns; ++j) {
    TRY(launch_operator_batched(L, OP_CHEB, nrhs, ld, cur, oth, b, j == 1 && x0_zero ? nullptr : oth, sig[j], th[j],
                                nullptr, s, fe));
    std::swap(cur, oth);
  }
  if (cur != x) return fail(HMG_ERR_INVALID, "internal: Chebyshev buffer parity");
  return HMG_OK;
}

// r_q = b_q - A x_q for nrhs vectors
static int residual_v(const hmg_level* L, int nrhs, int64_t ld, const void* x, void* r, const void* b, void* fe,
                      hipStream_t s) {
  if (L->space == HMG_DG || fe)
    return launch_operator_batched(L, OP_RESID, nrhs, ld, x, r, b, nullptr, 0, 0, nullptr, s, fe);
  const size_t o = ld * L->elem_size();
  for (int q = 0; q < nrhs; ++q)
    TRY(launch_operator(L, OP_RESID, (const char*)x + q * o, (char*)r + q * o, (const char*)b + q * o, nullptr, 0, 0,
                        nullptr, s));
  return HMG_OK;
}

// Coarsest level of the several-vector V-cycle: each vector by the selected
// coarse solve (exact, smoothing only or the FP64 iterative solve).
static int coarse_v(hmg_hierarchy* H, size_t l, int nrhs, hipStream_t s) {
  hmg_level* L = H->lv[l];
  const int64_t ld = H->ldl[l];
  const size_t o = ld * L->elem_size();
  int* skip = (int*)(H->scal() + 24);
  for (int q = 0; q < nrhs; ++q) {
    const void* b = (const char*)H->bb(l) + q * o;
    void* x = (char*)H->xb(l) + q * o;
    if (H->cap_buf && H->cap_count < H->cap_capacity) {  // training data (hmg_hierarchy_capture)
      TRY(vec_convert(L->prec, b, HMG_F64, H->cap_buf + (size_t)H->cap_count * H->nc, H->nc, s));
      H->cap_count++;
    }
    switch (H->coarse_mode) {
      case HMG_COARSE_SMOOTH:
        TRY(chebyshev(L, b, x, H->ns, H->lmax_c, 0.06, 1.2, 1, s));
        break;
      case HMG_COARSE_CG:
        TRY(set_flag(skip, 0, s));
        if (H->own_coarse64) TRY(set_flag(skip + 2, 0, s));
        TRY(coarse_cg64_at(H, l, b, x, s));
        break;
      case HMG_COARSE_EXACT:
        TRY(coarse_gemv(L->prec, H->ainv(), b, x, (int)H->nc, s));
        break;
      default:
        return fail(HMG_ERR_UNSUPPORTED, "several right-hand sides: exact, iterative or smoothing coarse solve");
    }
  }
  return HMG_OK;
}

// Transfers of nrhs vectors, one launch per kernel: vector q of the fine
// block q * ldf values on, of the coarse block q * ldc values on.  sf, sc:
// element-local blocks of the fine and coarse levels (n_dg values per
// vector), needed by the p- and h-transfers of continuous FE levels.
static int restrict_v(const hmg_transfer* T, int nrhs, const void* fine, int64_t ldf, void* coarse, int64_t ldc,
                      void* sf, void* sc, hipStream_t s) {
  const hmg_level *F = T->f, *C = T->c;
  const int pr = F->prec;
  if (T->kind == 'c') return tr_c_sum(pr, F->mesh, F->k, fine, coarse, 0, 0, s, nrhs, ldf, ldc);
  const int kind = T->kind == 'h' ? 1 : 0;
  const double* P1 = T->P1.empty() ? nullptr : T->P1.data();
  if (!T->fe)
    return tr_dg_restrict(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, fine, coarse, s, nrhs, ldf, ldc);
  if (!sf || !sc) return fail(HMG_ERR_INVALID, "internal: FE transfer without element-local blocks");
  TRY(tr_c_inject(pr, F->mesh, F->k, fine, sf, 1, 0, s, nrhs, ldf, F->n_dg));
  TRY(tr_dg_restrict(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, sf, sc, s, nrhs, F->n_dg, C->n_dg));
  return tr_c_sum(pr, C->mesh, C->k, sc, coarse, 0, 0, s, nrhs, C->n_dg, ldc);
}
static int prolongate_add_v(const hmg_transfer* T, int nrhs, const void* coarse, int64_t ldc, void* fine, int64_t ldf,
                            void* sf, void* sc, hipStream_t s) {
  const hmg_level *F = T->f, *C = T->c;
  const int pr = F->prec;
  if (T->kind == 'c') return tr_c_inject(pr, F->mesh, F->k, coarse, fine, 0, 1, s, nrhs, ldc, ldf);
  const int kind = T->kind == 'h' ? 1 : 0;
  const double* P1 = T->P1.empty() ? nullptr : T->P1.data();
  if (!T->fe)
    return tr_dg_prolongate(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, coarse, fine, 1, s, nrhs, ldc, ldf);
  if (!sf || !sc) return fail(HMG_ERR_INVALID, "internal: FE transfer without element-local blocks");
  TRY(tr_c_inject(pr, C->mesh, C->k, coarse, sc, 0, 0, s, nrhs, ldc, C->n_dg));
  TRY(tr_dg_prolongate(pr, kind, F->n, C->n, F->mesh.N, T->P0.data(), P1, sc, sf, 0, s, nrhs, C->n_dg, F->n_dg));
  return tr_c_sum(pr, F->mesh, F->k, sf, fine, 1, 1, s, nrhs, F->n_dg, ldf);
}

// Alg. 2 on level l for the blocks bb(l) -> xb(l), nrhs vectors.
static int vcycle_v(hmg_hierarchy* H, size_t l, int nrhs, hipStream_t s) {
  hmg_level* L = H->lv[l];
  if (l + 1 == H->lv.size()) return coarse_v(H, l, nrhs, s);
  const int64_t ld = H->ldl[l], ldc = H->ldl[l + 1];
  TRY(chebyshev_v(L, nrhs, ld, H->bb(l), H->xb(l), H->tb(l), H->ns, H->lmax[l], 1, H->sb(l), s));
  TRY(residual_v(L, nrhs, ld, H->xb(l), H->rb(l), H->bb(l), H->sb(l), s));
  // the element-local blocks of both levels are free during the transfers
  TRY(restrict_v(H->tr[l], nrhs, H->rb(l), ld, H->bb(l + 1), ldc, H->sb(l), H->sb(l + 1), s));
  TRY(vcycle_v(H, l + 1, nrhs, s));
  TRY(prolongate_add_v(H->tr[l], nrhs, H->xb(l + 1), ldc, H->xb(l), ld, H->sb(l), H->sb(l + 1), s));
  // post-smoothing: the residual block is free again and serves as the third buffer
  return chebyshev_v(L, nrhs, ld, H->bb(l), H->xb(l), H->tb(l), H->ns, H->lmax[l], 0, H->sb(l), s, H->rb(l));
}

// z_q = M^{-1} r_q (FP64 blocks, ldr and ldz values apart).
static int precondition_v(hmg_hierarchy* H, int nrhs, const double* r, int64_t ldr, double* z, int64_t ldz,
                          hipStream_t s) {
  const int pr = H->mg_prec;
  const int64_t n = H->lv[0]->n_dofs;
  TRY(vec_convert_b(HMG_F64, r, ldr, pr, H->bb(0), H->ldl[0], n, nrhs, s));
  TRY(vcycle_v(H, 0, nrhs, s));
  return vec_convert_b(pr, H->xb(0), H->ldl[0], HMG_F64, z, ldz, n, nrhs, s);
}

static int check_rhs_block(const hmg_hierarchy* H, int nrhs, int64_t ld) {
  if (!H || !H->bound) return fail(HMG_ERR_WORKSPACE, "hierarchy missing or not bound");
  // without a reservation the vectors are solved one after another
  if (nrhs < 1 || nrhs > (H->max_rhs > 1 ? H->max_rhs : kMaxRhs))
    return fail(HMG_ERR_INVALID, "nrhs must be 1..max_rhs (hmg_hierarchy_set_max_rhs before bind)");
  if (ld < H->fine64->n_dofs || (ld * 8) % 256) return fail(HMG_ERR_INVALID, "ld must be >= n_dofs, ld * 8 a multiple of 256");
  if (nrhs > 1 && H->coarse_mode == HMG_COARSE_LEARNED)
    return fail(HMG_ERR_UNSUPPORTED, "several right-hand sides with the learned coarse solve");
  return HMG_OK;
}

extern "C" int hmg_hierarchy_set_max_rhs(hmg_hierarchy* H, int max_rhs) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (H->bound) return fail(HMG_ERR_INVALID, "set the number of right-hand sides before bind");
  if (max_rhs < 1 || max_rhs > kMaxRhs) return fail(HMG_ERR_INVALID, "max_rhs must be 1..64");
  H->max_rhs = max_rhs;
  hierarchy_layout(H);
  return HMG_OK;
}

extern "C" int hmg_vcycle_batched(hmg_hierarchy* H, int nrhs, const double* b, double* x, int64_t ld, hipStream_t s) {
  TRY(check_rhs_block(H, nrhs, ld));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(x, "x"));
  if (ranges_overlap(b, x, (size_t)(ld * (nrhs - 1) + H->fine64->n_dofs) * 8))
    return fail(HMG_ERR_INVALID, "b and x must not overlap");
  if (nrhs == 1 || H->max_rhs == 1) {
    for (int q = 0; q < nrhs; ++q) TRY(precondition(H, b + q * ld, x + q * ld, s));
    return HMG_OK;
  }
  return precondition_v(H, nrhs, b, ld, x, ld, s);
}

extern "C" int hmg_pcg_solve_batched(hmg_hierarchy* H, int nrhs, const double* b, double* x, int64_t ld, double rtol,
                                     double atol, int maxit, hmg_solve_stats* st, hipStream_t s) {
  TRY(check_rhs_block(H, nrhs, ld));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(x, "x"));
  if (maxit < 0) return fail(HMG_ERR_INVALID, "maxit < 0");
  if (ranges_overlap(b, x, (size_t)(ld * (nrhs - 1) + H->fine64->n_dofs) * 8))
    return fail(HMG_ERR_INVALID, "b and x must not overlap");
  if (nrhs == 1 || H->max_rhs == 1) {  // one at a time
    int worst = HMG_OK;
    for (int q = 0; q < nrhs; ++q) {
      const int rc = hmg_pcg_solve(H, b + q * ld, x + q * ld, rtol, atol, maxit, st ? st + q : nullptr, s);
      if (rc < 0) return rc;
      worst = std::max(worst, rc);
    }
    return worst;
  }
  const hmg_level* A = H->fine64;
  const int64_t n = A->n_dofs, L = H->ld64;
  // the caller's blocks serve directly when their stride is the internal one
  // (x is then updated in place); otherwise they are copied in and x out
  const bool own = ld != L;
  const double* const B = own ? H->cgb(0) : b;
  double* const X = own ? H->cgb(1) : x;
  double *R = H->cgb(2), *P = H->cgb(3), *V = H->cgb(4), *Z = H->cgb(5);
  // scalars per vector: 0 previous delta, 1 delta = r.z, 2 p.Ap, 3 r.r, 4 z.Ap, 5 omega
  double *s0 = H->scalb(0), *s1 = H->scalb(1), *s2 = H->scalb(2), *s3 = H->scalb(3), *s4 = H->scalb(4);
  double* const alpha = H->scalb(5);  // omega of each vector's deferred x step
  double* part = H->partb();
  int* act = H->actb();
  std::vector<hmg_solve_stats> stats(nrhs, hmg_solve_stats{0, 0, 0, 0, 0});
  std::vector<int> active(nrhs, 1);
  std::vector<double> r0(nrhs), hs(2 * nrhs);
  auto finish = [&](int code) {
    for (int q = 0; q < nrhs; ++q) {
      if (stats[q].iters > 0 && stats[q].r0 > 0) {
        stats[q].rho = std::pow(stats[q].rn / stats[q].r0, 1.0 / stats[q].iters);
        stats[q].n10 = -10.0 / std::log10(stats[q].rho);
      }
      if (st) st[q] = stats[q];
    }
    return code;
  };
  auto upload_active = [&]() -> int {
    HMG_HIP(hipMemcpyAsync(act, active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
    HMG_HIP(hipStreamSynchronize(s));
    return HMG_OK;
  };
  if (own) {
    TRY(vec_convert_b(HMG_F64, b, ld, HMG_F64, H->cgb(0), L, n, nrhs, s));
    TRY(vec_convert_b(HMG_F64, x, ld, HMG_F64, X, L, n, nrhs, s));
  }
  TRY(launch_operator_batched(A, OP_RESID, nrhs, L, X, R, B, nullptr, 0, 0, nullptr, s));
  TRY(vec_dot_b(R, R, n, L, nrhs, part, s3, s));
  HMG_HIP(hipMemcpyAsync(hs.data(), s3, nrhs * 8, hipMemcpyDeviceToHost, s));
  HMG_HIP(hipStreamSynchronize(s));
  int n_active = 0;
  for (int q = 0; q < nrhs; ++q) {
    r0[q] = std::sqrt(hs[q]);
    stats[q].r0 = stats[q].rn = r0[q];
    if (!std::isfinite(r0[q])) return finish(fail(HMG_ERR_NONFINITE, "initial residual is not finite"));
    active[q] = (r0[q] > 0 && r0[q] > atol) ? 1 : 0;
    n_active += active[q];
  }
  if (n_active == 0) return finish(HMG_OK);
  TRY(upload_active());
  // FP32 V-cycle inside standard CG: z stays in FP32 (see fp32_z)
  const bool zf = fp32_z(H);
  float* const r32 = zf ? (float*)H->bb(0) : nullptr;
  const float* const z32 = zf ? (const float*)H->xb(0) : nullptr;
  const int64_t l32 = H->ldl[0];
  if (zf) {
    TRY(vec_convert_b(HMG_F64, R, L, HMG_F32, r32, l32, n, nrhs, s));
    TRY(vcycle_v(H, 0, nrhs, s));
    TRY(cg_update_p_zf_b(P, z32, nullptr, nullptr, n, L, l32, nrhs, act, s));
    TRY(vec_dot_zf_b(R, z32, n, L, l32, nrhs, part, s1, s));
  } else {
    TRY(precondition_v(H, nrhs, R, L, Z, L, s));
    TRY(vec_copy(HMG_F64, Z, P, L * nrhs, s));
    TRY(vec_dot_b(R, Z, n, L, nrhs, part, s1, s));
  }
  int it = 0;
  while (n_active > 0 && it < maxit) {
    if (it > 0) {
      if (zf) {
        TRY(vcycle_v(H, 0, nrhs, s));  // the right-hand side block holds r in FP32 (cg_update_xr_b)
        TRY(vec_dot_zf_b(R, z32, n, L, l32, nrhs, part, s1, s));
        // also takes the last update's deferred step x += alpha p
        TRY(cg_update_p_zf_b(P, z32, s1, s0, n, L, l32, nrhs, act, s, X, alpha));
      } else {
        TRY(precondition_v(H, nrhs, R, L, Z, L, s));
        TRY(vec_dot_b(R, Z, n, L, nrhs, part, s1, s));
        if (H->flexible) {
          TRY(vec_dot_b(Z, V, n, L, nrhs, part, s4, s));
          TRY(cg_update_p_b(P, Z, s4, s2, n, L, nrhs, act, true, s));
        } else {
          TRY(cg_update_p_b(P, Z, s1, s0, n, L, nrhs, act, false, s));
        }
      }
    }
    if (double* const db = H->dotb()) {  // p.(A p) summed per work item by the apply
      TRY(launch_operator_batched(A, OP_DOT, nrhs, L, P, V, nullptr, nullptr, 0, 0, nullptr, s, db));
      TRY(reduce_strided(db, A->n_el, nrhs, s2, part, s));
    } else {
      TRY(launch_operator_batched(A, OP_APPLY, nrhs, L, P, V, nullptr, nullptr, 0, 0, nullptr, s));
      TRY(vec_dot_b(P, V, n, L, nrhs, part, s2, s));
    }
    // with the FP32 z the step x += alpha p waits for the next direction
    // update, which reads p anyway (one pass over p fewer)
    TRY(cg_update_xr_b(zf ? nullptr : X, R, P, V, s1, s2, n, L, nrhs, part, s3, s0, act, s, r32, l32, alpha));
    HMG_HIP(hipMemcpyAsync(hs.data(), s2, nrhs * 8, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipMemcpyAsync(hs.data() + nrhs, s3, nrhs * 8, hipMemcpyDeviceToHost, s));
    HMG_HIP(hipStreamSynchronize(s));
    ++it;
    bool changed = false;
    uint64_t live = 0, done = 0;  // vectors of this update; those that stop now
    for (int q = 0; q < nrhs; ++q)
      if (active[q]) live |= 1ull << q;
    for (int q = 0; q < nrhs; ++q) {
      if (!active[q]) continue;
      const double nr = std::sqrt(hs[nrhs + q]);
      stats[q].iters = it;
      stats[q].rn = nr;
      if (!(hs[q] > 0)) {
        if (zf) TRY(cg_step_x_b(X, P, alpha, n, L, nrhs, live, s));
        if (own) TRY(vec_convert_b(HMG_F64, X, L, HMG_F64, x, ld, n, nrhs, s));
        return finish(fail(HMG_ERR_BREAKDOWN, "p^T A p <= 0: operator not SPD"));
      }
      if (!std::isfinite(nr)) return finish(fail(HMG_ERR_NONFINITE, "residual is not finite"));
      if (!(nr / r0[q] > rtol && nr > atol)) {
        active[q] = 0;
        --n_active;
        changed = true;
        done |= 1ull << q;
      }
    }
    if (zf) TRY(cg_step_x_b(X, P, alpha, n, L, nrhs, done, s));  // their last step
    if (changed && n_active > 0) TRY(upload_active());
  }
  if (zf && it > 0) {  // the last step of the vectors still running (maxit reached)
    uint64_t live = 0;
    for (int q = 0; q < nrhs; ++q)
      if (active[q]) live |= 1ull << q;
    TRY(cg_step_x_b(X, P, alpha, n, L, nrhs, live, s));
  }
  if (own) TRY(vec_convert_b(HMG_F64, X, L, HMG_F64, x, ld, n, nrhs, s));
  HMG_HIP(hipStreamSynchronize(s));
  return finish(n_active > 0 ? HMG_NOT_CONVERGED : HMG_OK);
}

extern "C" int hmg_hierarchy_set_coarse(hmg_hierarchy* H, int mode, hmg_net* net, double accept) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (mode != HMG_COARSE_EXACT && mode != HMG_COARSE_SMOOTH && mode != HMG_COARSE_LEARNED &&
      mode != HMG_COARSE_CG)
    return fail(HMG_ERR_INVALID, "unknown coarse mode");
  if (mode == HMG_COARSE_EXACT && !H->dense)
    return fail(HMG_ERR_UNSUPPORTED, "no dense coarse inverse above 8192 unknowns");
  if (mode == HMG_COARSE_LEARNED) {
    if (!net || !net->bound) return fail(HMG_ERR_INVALID, "learned coarse solve needs a bound network");
    if (H->lv.back()->space != HMG_FE || H->lv.back()->k != 1)
      return fail(HMG_ERR_UNSUPPORTED, "learned coarse solve needs a continuous Q1 coarsest level");
    const NodeGrid ng = coarse_nodes(H);
    if (ng.Mx > net->G || ng.My > net->G || ng.Mz > net->G)
      return fail(HMG_ERR_UNSUPPORTED, "network grid smaller than the coarse node grid");
    if (!(accept > 0)) return fail(HMG_ERR_INVALID, "accept must be positive");
  }
  H->coarse_mode = mode;
  H->net = mode == HMG_COARSE_LEARNED ? net : nullptr;
  H->accept = accept;
  // an inexact or learned coarse solve changes the preconditioner between iterations
  H->flexible = (mode == HMG_COARSE_LEARNED || mode == HMG_COARSE_CG) ? true : H->flexible;
  H->drop_graphs();
  return HMG_OK;
}

extern "C" int hmg_hierarchy_set_flexible(hmg_hierarchy* H, int enable) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  H->flexible = enable != 0;
  H->drop_graphs();
  return HMG_OK;
}

extern "C" int hmg_hierarchy_coarse_info(const hmg_hierarchy* H, int64_t* n, int* Mx, int* My, int* Mz,
                                         double* scale) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (n) *n = H->nc;
  const hmg_level* C = H->lv.back();
  const bool fe = C->space == HMG_FE;
  if (Mx) *Mx = fe ? C->mesh.N[0] * C->k + 1 : 0;
  if (My) *My = fe ? C->mesh.N[1] * C->k + 1 : 0;
  if (Mz) *Mz = fe ? C->mesh.N[2] * C->k + 1 : 0;
  if (scale) *scale = H->c0;
  return HMG_OK;
}

extern "C" int hmg_hierarchy_capture(hmg_hierarchy* H, double* buf, int capacity) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (capacity < 0 || (capacity > 0 && !buf)) return fail(HMG_ERR_INVALID, "need a buffer for capacity > 0");
  if (buf) TRY(check_ptr(buf, "buf"));
  H->cap_buf = capacity > 0 ? buf : nullptr;
  H->cap_capacity = capacity;
  H->cap_count = 0;
  return HMG_OK;
}

extern "C" int hmg_hierarchy_captured(const hmg_hierarchy* H, int* count) {
  if (!H || !count) return fail(HMG_ERR_INVALID, "NULL argument");
  *count = H->cap_count;
  return HMG_OK;
}

extern "C" int hmg_hierarchy_coarse_solve_batch(const hmg_hierarchy* H, const double* R, double* E, int count,
                                                hipStream_t s) {
  if (!H || !H->bound) return fail(HMG_ERR_WORKSPACE, "hierarchy missing or not bound");
  if (count < 0) return fail(HMG_ERR_INVALID, "count < 0");
  if (count == 0) return HMG_OK;
  TRY(check_ptr(R, "R"));
  TRY(check_ptr(E, "E"));
  {
    const size_t len = (size_t)count * H->nc;
    if (R < E + len && E < R + len) return fail(HMG_ERR_INVALID, "R and E must not overlap");
  }
  if (H->dense) return coarse_gemm(H->ainv(), R, E, (int)H->nc, count, s);
  // no dense inverse: FP64 Jacobi-PCG on the FP64 coarse level, sample by sample
  hmg_hierarchy* Hm = const_cast<hmg_hierarchy*>(H);
  int* skip = (int*)(H->scal() + 24);
  for (int i = 0; i < count; ++i) {
    TRY(set_flag(skip, 0, s));
    TRY(coarse_cg(Hm, H->coarse64, R + (size_t)i * H->nc, E + (size_t)i * H->nc, 1e-12, 20000, s));
  }
  return HMG_OK;
}

extern "C" int hmg_hierarchy_learned_data(const hmg_hierarchy* H, int grid, const double* R, const double* E,
                                          int count, float* in, float* target, hipStream_t s) {
  if (!H || !H->bound) return fail(HMG_ERR_WORKSPACE, "hierarchy missing or not bound");
  const hmg_level* C = H->lv.back();
  if (C->space != HMG_FE || C->k != 1) return fail(HMG_ERR_UNSUPPORTED, "needs a continuous Q1 coarsest level");
  const NodeGrid ng = coarse_nodes(H);
  if (grid < ng.Mx || grid < ng.My || grid < ng.Mz) return fail(HMG_ERR_INVALID, "grid smaller than the node grid");
  if (count < 1) return fail(HMG_ERR_INVALID, "count < 1");
  TRY(check_ptr(R, "R"));
  TRY(check_ptr(in, "in"));
  if (target) {
    TRY(check_ptr(E, "E"));
  }
  // per-sample sigma in the caller's input buffer would clash: use the
  // hierarchy's reduction scratch (count <= kPartials samples per call)
  if (count > kPartials) return fail(HMG_ERR_INVALID, "at most 1024 samples per call");
  return net_pack(HMG_F64, R, target ? E : nullptr, H->nc, count, ng, grid, H->c0, H->part(), in, target, s);
}

extern "C" int hmg_hierarchy_coarse_stats(const hmg_hierarchy* H, int* fallbacks, hipStream_t s) {
  if (!H || !H->bound || !fallbacks) return fail(HMG_ERR_INVALID, "hierarchy not bound or NULL argument");
  HMG_HIP(hipMemcpyAsync(fallbacks, H->scal() + 10, sizeof(int), hipMemcpyDeviceToHost, s));
  HMG_HIP(hipStreamSynchronize(s));
  return HMG_OK;
}

extern "C" int hmg_hierarchy_set_coarse_cg(hmg_hierarchy* H, double rtol, int maxit) {
  if (!H) return fail(HMG_ERR_INVALID, "hierarchy is NULL");
  if (!(rtol > 0) || !(rtol < 1) || maxit < 1 || maxit > 100000)
    return fail(HMG_ERR_INVALID, "need 0 < rtol < 1 and 1 <= maxit <= 100000");
  H->coarse_rtol = rtol;
  H->coarse_maxit = maxit;
  H->drop_graphs();
  return HMG_OK;
}
