// Host-side setup: 1-D bases, the Q3 element mapping, geometric factors,
// penalty parameters and the manufactured right-hand side.  None of this
// is timed (Sec. 3.1: setup costs are excluded from the cost measures).
#include <algorithm>
#include <cmath>
#include <thread>

#include "hmg_internal.h"

namespace hmg {

// ------------------------------------------------------------------ 1-D bases
// Legendre P_m(t), P_m'(t) by the three-term recurrence.
static void legendre(int m, double t, double& P, double& dP) {
  double p0 = 1.0, p1 = t;
  if (m == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int j = 1; j < m; ++j) {
    double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = m * (p0 - t * p1) / (1.0 - t * t);  // valid for |t| < 1
}

// GLL nodes of degree k on [0,1]: end points and the roots of P_k', found by
// Newton's method with P_k'' from Legendre's differential equation.
std::vector<double> gll_nodes(int k) {
  std::vector<double> x(k + 1);
  x[0] = -1.0;
  x[k] = 1.0;
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(M_PI * j / k);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(k, t, P, dP);
      double d2P = (2.0 * t * dP - k * (k + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[j] = t;
  }
  std::sort(x.begin(), x.end());
  for (auto& v : x) v = 0.5 * (v + 1.0);
  x[0] = 0.0;
  x[k] = 1.0;
  return x;
}

// n-point Gauss-Legendre rule on [0,1] by Newton's method on P_n.
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double t = std::cos(M_PI * (j + 0.75) / (n + 0.5));
    double P = 0, dP = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(n, t, P, dP);
      double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre(n, t, P, dP);
    x[n - 1 - j] = 0.5 * (t + 1.0);
    w[n - 1 - j] = 1.0 / ((1.0 - t * t) * dP * dP);  // 2/((1-t^2)P'^2) / 2
  }
}

// Barycentric Lagrange interpolation: values and first derivatives.
void lagrange(const std::vector<double>& nodes, const std::vector<double>& x,
              std::vector<double>* V, std::vector<double>* Dv) {
  const int n = (int)nodes.size(), m = (int)x.size();
  std::vector<double> lam(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (j != i) lam[i] /= (nodes[i] - nodes[j]);
  if (V) V->assign((size_t)m * n, 0.0);
  if (Dv) Dv->assign((size_t)m * n, 0.0);
  for (int q = 0; q < m; ++q) {
    int hit = -1;
    for (int i = 0; i < n; ++i)
      if (x[q] == nodes[i]) hit = i;
    if (hit >= 0) {
      if (V) (*V)[(size_t)q * n + hit] = 1.0;
      if (Dv) {
        double diag = 0.0;
        for (int i = 0; i < n; ++i) {
          if (i == hit) continue;
          double d = (lam[i] / lam[hit]) / (nodes[hit] - nodes[i]);
          (*Dv)[(size_t)q * n + i] = d;
          diag -= d;
        }
        (*Dv)[(size_t)q * n + hit] = diag;
      }
      continue;
    }
    double den = 0.0;
    for (int i = 0; i < n; ++i) den += lam[i] / (x[q] - nodes[i]);
    for (int i = 0; i < n; ++i) {
      double li = (lam[i] / (x[q] - nodes[i])) / den;
      if (V) (*V)[(size_t)q * n + i] = li;
      if (Dv) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
          if (j != i) s += 1.0 / (x[q] - nodes[j]);
        (*Dv)[(size_t)q * n + i] = li * s;
      }
    }
  }
}

Basis1D make_basis(int k) {
  Basis1D b;
  b.k = k;
  b.n = k + 1;
  const int n = b.n;
  b.gll = gll_nodes(k);
  gauss_rule(n, b.gz, b.gw);
  lagrange(b.gll, b.gz, &b.S, &b.Sp);
  lagrange(b.gz, b.gz, nullptr, &b.D);
  b.M.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += b.gw[q] * b.S[q * n + i] * b.S[q * n + j];
      b.M[i * n + j] = s;
    }
  b.K.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += b.gw[q] * b.Sp[q * n + i] * b.Sp[q * n + j];
      b.K[i * n + j] = s;
    }
  std::vector<double> Dend, Gend;
  lagrange(b.gll, {0.0, 1.0}, nullptr, &Dend);
  b.dl0.assign(Dend.begin(), Dend.begin() + n);
  b.dl1.assign(Dend.begin() + n, Dend.end());
  lagrange(b.gz, {0.0, 1.0}, &Gend, nullptr);
  b.lg0.assign(Gend.begin(), Gend.begin() + n);
  b.lg1.assign(Gend.begin() + n, Gend.end());
  return b;
}

// Even-odd packing (sig = +1 centrosymmetric, -1 skew): see TabOff.
static void eo_pack(const std::vector<double>& A, int n, std::vector<double>& out) {
  const int h = n / 2;
  for (int q = 0; q < h; ++q)
    for (int i = 0; i < h; ++i) out.push_back(0.5 * (A[q * n + i] + A[q * n + n - 1 - i]));
  for (int q = 0; q < h; ++q)
    for (int i = 0; i < h; ++i) out.push_back(0.5 * (A[q * n + i] - A[q * n + n - 1 - i]));
  if (n & 1) {
    for (int q = 0; q < h; ++q) out.push_back(A[q * n + h]);
    for (int i = 0; i < h; ++i) out.push_back(A[h * n + i]);
    out.push_back(A[h * n + h]);
  }
}

static std::vector<double> transpose(const std::vector<double>& A, int n) {
  std::vector<double> T((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[j * n + i] = A[i * n + j];
  return T;
}

std::vector<double> op_tables(const Basis1D& b) {
  const int n = b.n;
  std::vector<double> t;
  t.insert(t.end(), b.S.begin(), b.S.end());
  t.insert(t.end(), b.Sp.begin(), b.Sp.end());
  t.insert(t.end(), b.M.begin(), b.M.end());
  t.insert(t.end(), b.dl0.begin(), b.dl0.end());
  t.insert(t.end(), b.dl1.begin(), b.dl1.end());
  t.insert(t.end(), b.lg0.begin(), b.lg0.end());
  t.insert(t.end(), b.lg1.begin(), b.lg1.end());
  eo_pack(b.S, n, t);
  eo_pack(transpose(b.S, n), n, t);
  eo_pack(transpose(b.Sp, n), n, t);
  eo_pack(b.D, n, t);
  eo_pack(b.M, n, t);
  eo_pack(b.K, n, t);
  return t;
}

// ------------------------------------------------------------------ mapping
static const std::vector<double>& q3_nodes() {
  static const std::vector<double> g = gll_nodes(3);
  return g;
}

// Q3 support points of element e (Sec. 5.3: cubic mapping), X[(a+4b+16c)*3+r].
static void support_points(const Mesh& m, int64_t e, double X[192]) {
  const auto& g = q3_nodes();
  int64_t ex = e % m.N[0], ey = (e / m.N[0]) % m.N[1], ez = e / ((int64_t)m.N[0] * m.N[1]);
  int64_t ec[3] = {ex, ey, ez};
  for (int c = 0; c < 4; ++c)
    for (int b = 0; b < 4; ++b)
      for (int a = 0; a < 4; ++a) {
        int idx[3] = {a, b, c};
        double p[3], s[3];
        for (int d = 0; d < 3; ++d) {
          p[d] = m.lo[d] + (ec[d] + g[idx[d]]) * m.h(d);
          s[d] = (p[d] - m.lo[d]) / (m.hi[d] - m.lo[d]);
        }
        double bump = 0.0;
        if (m.curved)
          bump = m.amp * std::sin(m.waves * M_PI * s[0]) * std::sin(m.waves * M_PI * s[1]) *
                 std::sin(m.waves * M_PI * s[2]);
        for (int d = 0; d < 3; ++d) X[(a + 4 * b + 16 * c) * 3 + d] = p[d] + bump;
      }
}

// x and J (row-major J[r*3+s] = dx_r/dxi_s) on the tensor grid p0 x p1 x p2
// (first index fastest), by sum factorization of the Q3 map.
static void map_grid(const double X[192], const std::vector<double> pts[3], std::vector<double>& x,
                     std::vector<double>& J) {
  const auto& g = q3_nodes();
  std::vector<double> V[3], Dv[3];
  for (int d = 0; d < 3; ++d) lagrange(g, pts[d], &V[d], &Dv[d]);
  const int n0 = (int)pts[0].size(), n1 = (int)pts[1].size(), n2 = (int)pts[2].size();
  // contract c -> q2: Y[a][b][q2][r], dY (d/dxi_2)
  std::vector<double> Y(4 * 4 * n2 * 3, 0.0), dY(4 * 4 * n2 * 3, 0.0);
  for (int q2 = 0; q2 < n2; ++q2)
    for (int b = 0; b < 4; ++b)
      for (int a = 0; a < 4; ++a)
        for (int r = 0; r < 3; ++r) {
          double s = 0, ds = 0;
          for (int c = 0; c < 4; ++c) {
            double v = X[(a + 4 * b + 16 * c) * 3 + r];
            s += V[2][q2 * 4 + c] * v;
            ds += Dv[2][q2 * 4 + c] * v;
          }
          Y[((a * 4 + b) * n2 + q2) * 3 + r] = s;
          dY[((a * 4 + b) * n2 + q2) * 3 + r] = ds;
        }
  // contract b -> q1: Z (value), Zy (d/dxi_1), Zz (d/dxi_2)
  std::vector<double> Z(4 * n1 * n2 * 3), Zy(4 * n1 * n2 * 3), Zz(4 * n1 * n2 * 3);
  for (int q2 = 0; q2 < n2; ++q2)
    for (int q1 = 0; q1 < n1; ++q1)
      for (int a = 0; a < 4; ++a)
        for (int r = 0; r < 3; ++r) {
          double s = 0, sy = 0, sz = 0;
          for (int b = 0; b < 4; ++b) {
            double y = Y[((a * 4 + b) * n2 + q2) * 3 + r];
            s += V[1][q1 * 4 + b] * y;
            sy += Dv[1][q1 * 4 + b] * y;
            sz += V[1][q1 * 4 + b] * dY[((a * 4 + b) * n2 + q2) * 3 + r];
          }
          size_t o = ((a * n1 + q1) * n2 + q2) * 3 + r;
          Z[o] = s;
          Zy[o] = sy;
          Zz[o] = sz;
        }
  const int np = n0 * n1 * n2;
  x.assign((size_t)np * 3, 0.0);
  J.assign((size_t)np * 9, 0.0);
  for (int q2 = 0; q2 < n2; ++q2)
    for (int q1 = 0; q1 < n1; ++q1)
      for (int q0 = 0; q0 < n0; ++q0) {
        int p = q0 + n0 * (q1 + n1 * q2);
        for (int r = 0; r < 3; ++r) {
          double s = 0, s0 = 0, s1 = 0, s2 = 0;
          for (int a = 0; a < 4; ++a) {
            size_t o = ((a * n1 + q1) * n2 + q2) * 3 + r;
            s += V[0][q0 * 4 + a] * Z[o];
            s0 += Dv[0][q0 * 4 + a] * Z[o];
            s1 += V[0][q0 * 4 + a] * Zy[o];
            s2 += V[0][q0 * 4 + a] * Zz[o];
          }
          x[p * 3 + r] = s;
          J[p * 9 + r * 3 + 0] = s0;
          J[p * 9 + r * 3 + 1] = s1;
          J[p * 9 + r * 3 + 2] = s2;
        }
      }
}

// x and J of the analytic map (the undeformed point plus the deformation;
// J = diag(h) + gradient of the deformation, ds_d/dxi_d = 1/N_d) on the
// tensor grid pts (first index fastest).
static void exact_grid(const Mesh& m, int64_t e, const std::vector<double> pts[3], std::vector<double>& x,
                       std::vector<double>& J) {
  const int64_t ec[3] = {e % m.N[0], (e / m.N[0]) % m.N[1], e / ((int64_t)m.N[0] * m.N[1])};
  const int n0 = (int)pts[0].size(), n1 = (int)pts[1].size(), n2 = (int)pts[2].size();
  x.assign((size_t)n0 * n1 * n2 * 3, 0.0);
  J.assign((size_t)n0 * n1 * n2 * 9, 0.0);
  const double w = m.waves * M_PI;
  for (int q2 = 0; q2 < n2; ++q2)
    for (int q1 = 0; q1 < n1; ++q1)
      for (int q0 = 0; q0 < n0; ++q0) {
        const int p = q0 + n0 * (q1 + n1 * q2);
        const double xi[3] = {pts[0][q0], pts[1][q1], pts[2][q2]};
        double pt[3], sn[3], cs[3];
        for (int d = 0; d < 3; ++d) {
          pt[d] = m.lo[d] + (ec[d] + xi[d]) * m.h(d);
          const double sd = (pt[d] - m.lo[d]) / (m.hi[d] - m.lo[d]);
          sn[d] = std::sin(w * sd);
          cs[d] = std::cos(w * sd);
        }
        const double bump = m.curved ? m.amp * sn[0] * sn[1] * sn[2] : 0.0;
        for (int r = 0; r < 3; ++r) {
          x[p * 3 + r] = pt[r] + bump;
          J[p * 9 + r * 3 + r] = m.h(r);
        }
        if (m.curved)
          for (int c = 0; c < 3; ++c) {
            const double db = m.amp * w * cs[c] * sn[(c + 1) % 3] * sn[(c + 2) % 3] / m.N[c];
            for (int r = 0; r < 3; ++r) J[p * 9 + r * 3 + c] += db;
          }
      }
}

// The map of element e: the Q3 interpolant of the deformation (Sec. 5.3:
// cubic mapping) or, with mapping degree 0, the deformation itself.
struct ElemMap {
  const Mesh& m;
  int64_t e;
  double X[192];
  ElemMap(const Mesh& mesh, int64_t el) : m(mesh), e(el) {
    if (m.mapdeg != 0) support_points(m, e, X);
  }
  void grid(const std::vector<double> pts[3], std::vector<double>& x, std::vector<double>& J) const {
    if (m.mapdeg != 0) map_grid(X, pts, x, J);
    else exact_grid(m, e, pts, x, J);
  }
};

void map_point(const Mesh& m, int64_t e, const double xi[3], double x[3], double J[9]) {
  const ElemMap X(m, e);
  std::vector<double> pts[3] = {{xi[0]}, {xi[1]}, {xi[2]}}, xs, Js;
  X.grid(pts, xs, Js);
  for (int r = 0; r < 3; ++r) x[r] = xs[r];
  for (int r = 0; r < 9; ++r) J[r] = Js[r];
}

// inverse and determinant of a row-major 3x3 matrix
static double inv3(const double* A, double* B) {
  double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8],
         c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  double id = 1.0 / det;
  B[0] = c00 * id;
  B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = c01 * id;
  B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = c02 * id;
  B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return det;
}

template <typename F>
static void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64) nt = 1;
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &f] {
      for (int64_t i = a; i < b; ++i) f(i);
    });
  }
  for (auto& t : th) t.join();
}

static void face_pts(const Basis1D& b, int d, int s, std::vector<double> pts[3]) {
  for (int r = 0; r < 3; ++r) pts[r] = b.gz;
  pts[d] = {double(s)};
}

// Surface weight |det J| |J^{-T} n_ref| w_a w_b and outward unit normal at
// each face point from the element's own mapping (Nanson's formula).
static void face_normals(const std::vector<double>& J, const Basis1D& b, int d, int s,
                         std::vector<double>& nrm, std::vector<double>& dA,
                         std::vector<double>& Jinv) {
  const int n = b.n, nf = n * n;
  nrm.assign(nf * 3, 0.0);
  dA.assign(nf, 0.0);
  Jinv.assign(nf * 9, 0.0);
  double sg = s ? 1.0 : -1.0;
  for (int q = 0; q < nf; ++q) {
    double* Bi = &Jinv[q * 9];
    double det = inv3(&J[q * 9], Bi);
    double mv[3], nn = 0;
    for (int r = 0; r < 3; ++r) {
      mv[r] = sg * Bi[d * 3 + r];  // (J^{-T} n_ref)_r = sg * Jinv[d][r]
      nn += mv[r] * mv[r];
    }
    nn = std::sqrt(nn);
    int qa = q % n, qb = q / n;
    for (int r = 0; r < 3; ++r) nrm[q * 3 + r] = mv[r] / nn;
    dA[q] = std::fabs(det) * nn * b.gw[qa] * b.gw[qb];
  }
}

int build_geometry(const Mesh& m, const Basis1D& b, Geometry& g, bool faces) {
  const int n = b.n, n3 = n * n * n, nf = n * n;
  const int64_t ne = m.n_el();
  g.tau.assign(ne, 0.0);
  if (m.curved) g.metric.assign((size_t)ne * 6 * n3, 0.0);
  // cell metric, volume and tau
  parallel_for(ne, [&](int64_t e) {
    const ElemMap X(m, e);
    std::vector<double> pts[3] = {b.gz, b.gz, b.gz}, x, J;
    X.grid(pts, x, J);
    double vol = 0.0;
    for (int q = 0; q < n3; ++q) {
      double Bi[9];
      double det = inv3(&J[q * 9], Bi);
      int q0 = q % n, q1 = (q / n) % n, q2 = q / nf;
      double jxw = std::fabs(det) * b.gw[q0] * b.gw[q1] * b.gw[q2];
      vol += jxw;
      if (m.curved) {
        double G[3][3];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c)
            G[r][c] = jxw * (Bi[r * 3 + 0] * Bi[c * 3 + 0] + Bi[r * 3 + 1] * Bi[c * 3 + 1] +
                             Bi[r * 3 + 2] * Bi[c * 3 + 2]);
        double* o = &g.metric[(size_t)e * 6 * n3];
        o[0 * n3 + q] = G[0][0];
        o[1 * n3 + q] = G[1][1];
        o[2 * n3 + q] = G[2][2];
        o[3 * n3 + q] = G[0][1];
        o[4 * n3 + q] = G[0][2];
        o[5 * n3 + q] = G[1][2];
      }
    }
    int64_t ec[3] = {e % m.N[0], (e / m.N[0]) % m.N[1], e / ((int64_t)m.N[0] * m.N[1])};
    double area = 0.0;
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        std::vector<double> fp[3], fx, fJ, nrm, dA, Ji;
        face_pts(b, d, s, fp);
        X.grid(fp, fx, fJ);
        face_normals(fJ, b, d, s, nrm, dA, Ji);
        double a = 0.0;
        for (int q = 0; q < nf; ++q) a += dA[q];
        bool interior = s ? (ec[d] + 1 < m.N[d]) : (ec[d] > 0);
        area += interior ? 0.5 * a : a;
      }
    double sc = m.tau_scale.empty() ? 1.0 : m.tau_scale[e];
    g.tau[e] = m.ip * sc * (double)(n * n) * area / vol;
  });
  if (!m.curved || !faces) return HMG_OK;
  // face data: 3 directions, (N_d + 1) * N_a * N_b faces each
  for (int d = 0; d < 3; ++d) {
    int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
    int64_t nface = (int64_t)(m.N[d] + 1) * m.N[da] * m.N[db];
    g.face[d].assign((size_t)nface * 7 * nf, 0.0);
    parallel_for(nface, [&](int64_t f) {
      int p = (int)(f % (m.N[d] + 1));
      int64_t rest = f / (m.N[d] + 1);
      int ea = (int)(rest % m.N[da]), eb = (int)(rest / m.N[da]);
      auto elem = [&](int pd) {
        int c[3];
        c[d] = pd;
        c[da] = ea;
        c[db] = eb;
        return (int64_t)c[0] + (int64_t)m.N[0] * (c[1] + (int64_t)m.N[1] * c[2]);
      };
      double* o = &g.face[d][(size_t)f * 7 * nf];
      std::vector<double> nL, dAL, JiL, nR, dAR, JiR;
      bool hasL = p > 0, hasR = p < m.N[d];
      if (hasL) {
        const ElemMap X(m, elem(p - 1));
        std::vector<double> fp[3], fx, fJ;
        face_pts(b, d, 1, fp);
        X.grid(fp, fx, fJ);
        face_normals(fJ, b, d, 1, nL, dAL, JiL);
      }
      if (hasR) {
        const ElemMap X(m, elem(p));
        std::vector<double> fp[3], fx, fJ;
        face_pts(b, d, 0, fp);
        X.grid(fp, fx, fJ);
        face_normals(fJ, b, d, 0, nR, dAR, JiR);
      }
      for (int q = 0; q < nf; ++q) {
        double nv[3];
        for (int r = 0; r < 3; ++r) nv[r] = hasL ? nL[q * 3 + r] : -nR[q * 3 + r];
        o[6 * nf + q] = hasL ? dAL[q] : dAR[q];
        for (int sd = 0; sd < 3; ++sd) {
          // (n^T J^{-T})_sd = sum_r n_r Jinv[sd][r]
          if (hasL)
            o[sd * nf + q] = nv[0] * JiL[q * 9 + sd * 3 + 0] + nv[1] * JiL[q * 9 + sd * 3 + 1] +
                             nv[2] * JiL[q * 9 + sd * 3 + 2];
          if (hasR)
            o[(3 + sd) * nf + q] = nv[0] * JiR[q * 9 + sd * 3 + 0] +
                                   nv[1] * JiR[q * 9 + sd * 3 + 1] + nv[2] * JiR[q * 9 + sd * 3 + 2];
        }
      }
    });
  }
  return HMG_OK;
}

// b_i = (phi_i, f) - sum_{Dirichlet F} (dphi_i/dn - 2 tau phi_i, g)_F with
// u = prod sin(freq x_j), f = 3 freq^2 u, g = u (Sec. 2, inhomogeneous part
// of the mirror boundary conditions moved to the right-hand side).
int rhs_sine_host(const Mesh& m, const Basis1D& b, const Geometry& g, double freq,
                  std::vector<double>& out) {
  const int n = b.n, n3 = n * n * n, nf = n * n;
  const int64_t ne = m.n_el();
  out.assign((size_t)ne * n3, 0.0);
  auto uex = [&](const double* x) {
    return std::sin(freq * x[0]) * std::sin(freq * x[1]) * std::sin(freq * x[2]);
  };
  parallel_for(ne, [&](int64_t e) {
    const ElemMap X(m, e);
    std::vector<double> pts[3] = {b.gz, b.gz, b.gz}, x, J;
    X.grid(pts, x, J);
    std::vector<double> F(n3);
    for (int q = 0; q < n3; ++q) {
      double Bi[9];
      double det = inv3(&J[q * 9], Bi);
      int q0 = q % n, q1 = (q / n) % n, q2 = q / nf;
      F[q] = std::fabs(det) * b.gw[q0] * b.gw[q1] * b.gw[q2] * 3.0 * freq * freq * uex(&x[q * 3]);
    }
    double* o = &out[(size_t)e * n3];
    for (int l = 0; l < n; ++l)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int q2 = 0; q2 < n; ++q2)
            for (int q1 = 0; q1 < n; ++q1)
              for (int q0 = 0; q0 < n; ++q0)
                s += b.S[q0 * n + i] * b.S[q1 * n + j] * b.S[q2 * n + l] * F[q0 + n * (q1 + n * q2)];
          o[i + n * (j + n * l)] = s;
        }
    int64_t ec[3] = {e % m.N[0], (e / m.N[0]) % m.N[1], e / ((int64_t)m.N[0] * m.N[1])};
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        bool bnd = s ? (ec[d] + 1 == m.N[d]) : (ec[d] == 0);
        if (!bnd || m.bc[2 * d + s] != 0) continue;
        std::vector<double> fp[3], fx, fJ, nrm, dA, Ji;
        face_pts(b, d, s, fp);
        X.grid(fp, fx, fJ);
        face_normals(fJ, b, d, s, nrm, dA, Ji);
        int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
        for (int q = 0; q < nf; ++q) {
          int qa = q % n, qb = q / n;
          double c[3];
          for (int sd = 0; sd < 3; ++sd)
            c[sd] = nrm[q * 3 + 0] * Ji[q * 9 + sd * 3 + 0] + nrm[q * 3 + 1] * Ji[q * 9 + sd * 3 + 1] +
                    nrm[q * 3 + 2] * Ji[q * 9 + sd * 3 + 2];
          double gw = uex(&fx[q * 3]) * dA[q];
          for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
              for (int i = 0; i < n; ++i) {
                int idx[3] = {i, j, l};
                int pd = idx[d], ia = idx[da], ib = idx[db];
                double end_v = (pd == s * (n - 1)) ? 1.0 : 0.0;
                double end_d = s ? b.dl1[pd] : b.dl0[pd];
                double phi = end_v * b.S[qa * n + ia] * b.S[qb * n + ib];
                double gr[3];
                gr[d] = end_d * b.S[qa * n + ia] * b.S[qb * n + ib];
                gr[da] = end_v * b.Sp[qa * n + ia] * b.S[qb * n + ib];
                gr[db] = end_v * b.S[qa * n + ia] * b.Sp[qb * n + ib];
                double dphi = c[0] * gr[0] + c[1] * gr[1] + c[2] * gr[2];
                o[i + n * (j + n * l)] += gw * (2.0 * g.tau[e] * phi - dphi);
              }
        }
      }
  });
  return HMG_OK;
}

// diag(A) of a level from a(phi_i, phi_i) (Sec. 3.1: the diagonal of the
// Chebyshev-Jacobi smoother), evaluated on the host during setup.
// Cell part: sum_q sum_rs G_rs(q) d_r phi_i d_s phi_i, factorized per
// direction with the 1-D tables S^2, Sp^2 and S*Sp.  Face part (DG): only
// the n^2 nodes on a face plane have phi_i != 0 there; interior faces add
// tau phi^2 - phi dphi/dn, Dirichlet faces 2 tau phi^2 - 2 phi dphi/dn.
// FE: element cell diagonals summed over shared nodes, 1 on constrained nodes.
int diag_host(const Mesh& m, const Basis1D& b, const Geometry& g, int space,
              std::vector<double>& out) {
  const int n = b.n, n3 = n * n * n, nf = n * n;
  const int64_t ne = m.n_el();
  std::vector<double> A2(nf), B2(nf), C2(nf);  // [q][i]: S^2, Sp^2, S*Sp
  for (int i = 0; i < nf; ++i) {
    A2[i] = b.S[i] * b.S[i];
    B2[i] = b.Sp[i] * b.Sp[i];
    C2[i] = b.S[i] * b.Sp[i];
  }
  std::vector<double> local((size_t)ne * n3, 0.0);
  const double hx = m.h(0), hy = m.h(1), hz = m.h(2);
  const double cw[3] = {hy * hz / hx, hx * hz / hy, hx * hy / hz};
  parallel_for(ne, [&](int64_t e) {
    double* o = &local[(size_t)e * n3];
    // term (r, s): tables per direction
    const int comp_r[6] = {0, 1, 2, 0, 0, 1}, comp_s[6] = {0, 1, 2, 1, 2, 2};
    std::vector<double> G(n3), t1(n3), t2(n3);
    for (int c = 0; c < 6; ++c) {
      if (!m.curved && c >= 3) break;
      for (int q = 0; q < n3; ++q) {
        if (m.curved) {
          G[q] = g.metric[(size_t)e * 6 * n3 + (size_t)c * n3 + q] * (c >= 3 ? 2.0 : 1.0);
        } else {
          const int q0 = q % n, q1 = (q / n) % n, q2 = q / nf;
          G[q] = b.gw[q0] * b.gw[q1] * b.gw[q2] * cw[c];
        }
      }
      const double* T[3];
      for (int d = 0; d < 3; ++d) {
        const bool r = comp_r[c] == d, sd = comp_s[c] == d;
        T[d] = (r && sd) ? B2.data() : ((r || sd) ? C2.data() : A2.data());
      }
      // contract q0 -> i0, q1 -> i1, q2 -> i2
      for (int q2 = 0; q2 < n; ++q2)
        for (int q1 = 0; q1 < n; ++q1)
          for (int i0 = 0; i0 < n; ++i0) {
            double s = 0.0;
            for (int q0 = 0; q0 < n; ++q0) s += T[0][q0 * n + i0] * G[q0 + n * (q1 + n * q2)];
            t1[i0 + n * (q1 + n * q2)] = s;
          }
      for (int q2 = 0; q2 < n; ++q2)
        for (int i1 = 0; i1 < n; ++i1)
          for (int i0 = 0; i0 < n; ++i0) {
            double s = 0.0;
            for (int q1 = 0; q1 < n; ++q1) s += T[1][q1 * n + i1] * t1[i0 + n * (q1 + n * q2)];
            t2[i0 + n * (i1 + n * q2)] = s;
          }
      for (int i2 = 0; i2 < n; ++i2)
        for (int i1 = 0; i1 < n; ++i1)
          for (int i0 = 0; i0 < n; ++i0) {
            double s = 0.0;
            for (int q2 = 0; q2 < n; ++q2) s += T[2][q2 * n + i2] * t2[i0 + n * (i1 + n * q2)];
            o[i0 + n * (i1 + n * i2)] += s;
          }
    }
    if (space != HMG_DG) return;
    const int64_t ec[3] = {e % m.N[0], (e / m.N[0]) % m.N[1], e / ((int64_t)m.N[0] * m.N[1])};
    const double taue = g.tau[e];
    for (int d = 0; d < 3; ++d) {
      const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
      const int64_t stride = d == 0 ? 1 : (d == 1 ? (int64_t)m.N[0] : (int64_t)m.N[0] * m.N[1]);
      for (int s = 0; s < 2; ++s) {
        const bool has = s ? (ec[d] + 1 < m.N[d]) : (ec[d] > 0);
        if (!has && m.bc[2 * d + s] != 0) continue;  // homogeneous Neumann: 0
        const double tauF = has ? std::max(taue, g.tau[e + (s ? stride : -stride)]) : taue;
        const int pos = s * (n - 1);
        const double* dl = s ? b.dl1.data() : b.dl0.data();
        const double* fd = nullptr;
        if (m.curved) {
          const int Na = m.N[da];
          const int64_t f = (ec[d] + s) + (int64_t)(m.N[d] + 1) * (ec[da] + (int64_t)Na * ec[db]);
          fd = &g.face[d][(size_t)f * 7 * nf];
        }
        for (int ib = 0; ib < n; ++ib)
          for (int ia = 0; ia < n; ++ia) {
            int idx[3];
            idx[d] = pos;
            idx[da] = ia;
            idx[db] = ib;
            double acc = 0.0;
            for (int q = 0; q < nf; ++q) {
              const int qa = q % n, qb = q / n;
              const double sa = b.S[qa * n + ia], sb = b.S[qb * n + ib];
              double gr[3];
              gr[d] = dl[pos] * sa * sb;
              gr[da] = b.Sp[qa * n + ia] * sb;
              gr[db] = sa * b.Sp[qb * n + ib];
              const double phi = sa * sb;
              double co[3] = {0, 0, 0}, dA;
              if (m.curved) {
                for (int r = 0; r < 3; ++r) co[r] = s ? fd[r * nf + q] : -fd[(3 + r) * nf + q];
                dA = fd[6 * nf + q];
              } else {
                co[d] = (s ? 1.0 : -1.0) / m.h(d);
                dA = m.h(da) * m.h(db) * b.gw[qa] * b.gw[qb];
              }
              const double dphi = co[0] * gr[0] + co[1] * gr[1] + co[2] * gr[2];
              acc += has ? dA * (tauF * phi * phi - phi * dphi)
                         : dA * (2.0 * tauF * phi * phi - 2.0 * phi * dphi);
            }
            o[idx[0] + n * (idx[1] + n * idx[2])] += acc;
          }
      }
    }
  });
  if (space == HMG_DG) {
    out.swap(local);
    return HMG_OK;
  }
  // FE: sum over shared nodes; constrained nodes get 1
  const int k = b.k;
  const int64_t Mx = (int64_t)m.N[0] * k + 1, My = (int64_t)m.N[1] * k + 1, Mz = (int64_t)m.N[2] * k + 1;
  out.assign((size_t)(Mx * My * Mz), 0.0);
  for (int64_t e = 0; e < ne; ++e) {
    const int64_t ex = e % m.N[0], ey = (e / m.N[0]) % m.N[1], ez = e / ((int64_t)m.N[0] * m.N[1]);
    for (int l = 0; l < n; ++l)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          out[(ex * k + i) + Mx * ((ey * k + j) + My * (ez * k + l))] += local[(size_t)e * n3 + i + n * (j + n * l)];
  }
  for (int64_t gz = 0; gz < Mz; ++gz)
    for (int64_t gy = 0; gy < My; ++gy)
      for (int64_t gx = 0; gx < Mx; ++gx) {
        const bool fixed = (gx == 0 && !m.bc[0]) || (gx == Mx - 1 && !m.bc[1]) || (gy == 0 && !m.bc[2]) ||
                           (gy == My - 1 && !m.bc[3]) || (gz == 0 && !m.bc[4]) || (gz == Mz - 1 && !m.bc[5]);
        if (fixed) out[gx + Mx * (gy + My * gz)] = 1.0;
      }
  return HMG_OK;
}

}  // namespace hmg
