// Host construction: Gauss-Legendre operators, g_DG correction derivatives, curved-element
// metrics, geometric face matching (conforming and periodic) and probe location.
//
// FR (Huynh's scheme, named in the flow-solver subsection): the solution in an element is the
// Lagrange interpolant through the solution points; the flux derivative is corrected with the
// derivative of g_R = (P_{p+1} + P_p)/2 (1 at the right face, 0 at the left) and its mirror.
// Metric terms of the transformed conservation law (Eq. (1) on a curved element):
// A = dx/dxi, J = det A, S = J A^{-1} = adj(A); normals N = s_f S[k_f, :].
#include "fr_host.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <unordered_map>

#include "../../include/fr.h"

namespace frmi {
namespace {

// Legendre P_n and P_n' at x by the three-term recurrence and P'_{n+1} = P'_{n-1} + (2n+1) P_n.
void legendre(int n, double x, double &Pn, double &dPn) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { Pn = 1.0; dPn = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    double d2 = d0 + (2 * k + 1) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  Pn = p1; dPn = d1;
}

double lagrange_1d(const std::vector<double> &nodes, int b, double x) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != b) v *= (x - nodes[m]) / (nodes[b] - nodes[m]);
  return v;
}

double lagrange_1d_deriv(const std::vector<double> &nodes, int b, double x) {
  // derivative of the product by logarithmic differentiation written without division by (x - x_m)
  double s = 0.0;
  for (size_t r = 0; r < nodes.size(); ++r) {
    if ((int)r == b) continue;
    double t = 1.0 / (nodes[b] - nodes[r]);
    for (size_t m = 0; m < nodes.size(); ++m)
      if ((int)m != b && m != r) t *= (x - nodes[m]) / (nodes[b] - nodes[m]);
    s += t;
  }
  return s;
}

template <class F>
void parallel_for(int64_t n, F &&f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 256 || nt == 1) { for (int64_t i = 0; i < n; ++i) f(i); return; }
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> errs(nt);
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t] {
      try {
        for (int64_t i = (int64_t)t; i < n; i += nt) f(i);
      } catch (...) { errs[t] = std::current_exception(); }
    });
  }
  for (auto &x : th) x.join();
  for (auto &e : errs) if (e) std::rethrow_exception(e);
}

struct GeoBasis {
  int npts = 0, nn = 0;
  std::vector<double> phi;   // [npts][nn]
  std::vector<double> dphi;  // [dim][npts][nn]
};

GeoBasis geo_basis(int dim, int q, const std::vector<double> &ref /* [npts][dim] */) {
  std::vector<double> nodes = gll_nodes(q);
  int Q = q + 1;
  int nn = 1;
  for (int k = 0; k < dim; ++k) nn *= Q;
  GeoBasis b;
  b.npts = (int)(ref.size() / dim);
  b.nn = nn;
  b.phi.assign((size_t)b.npts * nn, 0.0);
  b.dphi.assign((size_t)dim * b.npts * nn, 0.0);
  for (int a = 0; a < b.npts; ++a) {
    for (int n = 0; n < nn; ++n) {
      int idx[3] = {n % Q, (n / Q) % Q, n / (Q * Q)};
      double lv[3], ld[3];
      for (int k = 0; k < dim; ++k) {
        lv[k] = lagrange_1d(nodes, idx[k], ref[a * dim + k]);
        ld[k] = lagrange_1d_deriv(nodes, idx[k], ref[a * dim + k]);
      }
      double v = 1.0;
      for (int k = 0; k < dim; ++k) v *= lv[k];
      b.phi[(size_t)a * nn + n] = v;
      for (int kd = 0; kd < dim; ++kd) {
        double dv = 1.0;
        for (int k = 0; k < dim; ++k) dv *= (k == kd ? ld[k] : lv[k]);
        b.dphi[((size_t)kd * b.npts + a) * nn + n] = dv;
      }
    }
  }
  return b;
}

// Reference coordinates of solution points (lexicographic, first fastest) and flux points
// (face f on coordinate f/2 at side -1/+1; tangential Gauss points lowest coordinate fastest).
std::vector<double> ref_solpts(int dim, const Ops1D &o) {
  int P = o.P, Ns = 1;
  for (int k = 0; k < dim; ++k) Ns *= P;
  std::vector<double> r((size_t)Ns * dim);
  for (int i = 0; i < Ns; ++i) {
    int ii[3] = {i % P, (i / P) % P, i / (P * P)};
    for (int k = 0; k < dim; ++k) r[(size_t)i * dim + k] = o.xi[ii[k]];
  }
  return r;
}

std::vector<double> ref_fpts(int dim, const Ops1D &o) {
  int P = o.P, Nfp = (dim == 2) ? P : P * P, Nf = 2 * dim * Nfp;
  std::vector<double> r((size_t)Nf * dim);
  for (int fp = 0; fp < Nf; ++fp) {
    int f = fp / Nfp, t = fp % Nfp, k = f / 2;
    double s = (f % 2) ? 1.0 : -1.0;
    int tt[2] = {t % P, t / P}, c = 0;
    for (int m = 0; m < dim; ++m) {
      if (m == k) r[(size_t)fp * dim + m] = s;
      else r[(size_t)fp * dim + m] = o.xi[tt[c++]];
    }
  }
  return r;
}

// x, A (A[j][k] = dx_j/dxi_k) at point a of a basis for element nodes Xe[nn][dim]
inline void map_point(int dim, const GeoBasis &b, int a, const double *Xe, double *x, double *A) {
  for (int j = 0; j < dim; ++j) {
    x[j] = 0.0;
    for (int k = 0; k < dim; ++k) A[j * dim + k] = 0.0;
  }
  const double *ph = &b.phi[(size_t)a * b.nn];
  for (int n = 0; n < b.nn; ++n)
    for (int j = 0; j < dim; ++j) x[j] += ph[n] * Xe[n * dim + j];
  for (int k = 0; k < dim; ++k) {
    const double *dp = &b.dphi[((size_t)k * b.npts + a) * b.nn];
    for (int n = 0; n < b.nn; ++n)
      for (int j = 0; j < dim; ++j) A[j * dim + k] += dp[n] * Xe[n * dim + j];
  }
}

// adj(A) (= J A^{-1}) and det A; adj[k*dim + j]
inline double adjugate(int dim, const double *A, double *adj) {
  if (dim == 2) {
    adj[0] = A[3]; adj[1] = -A[1];
    adj[2] = -A[2]; adj[3] = A[0];
    return A[0] * A[3] - A[1] * A[2];
  }
  double a[3][3];  // a[k] = column k
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) a[k][j] = A[j * 3 + k];
  auto cross = [](const double *u, const double *v, double *w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  cross(a[1], a[2], adj + 0);
  cross(a[2], a[0], adj + 3);
  cross(a[0], a[1], adj + 6);
  return adj[0] * a[0][0] + adj[1] * a[0][1] + adj[2] * a[0][2];
}

}  // namespace

std::vector<double> gll_nodes(int q) {
  switch (q) {
    case 1: return {-1.0, 1.0};
    case 2: return {-1.0, 0.0, 1.0};
    case 3: { double a = 1.0 / std::sqrt(5.0); return {-1.0, -a, a, 1.0}; }
    case 4: { double a = std::sqrt(3.0 / 7.0); return {-1.0, -a, 0.0, a, 1.0}; }
    default: throw FrError(FR_ERR_UNSUPPORTED, "geometry degree must be in 1..4");
  }
}

Ops1D build_ops_1d(int p) {
  Ops1D o;
  int P = p + 1;
  o.P = P;
  o.xi.resize(P);
  o.w.resize(P);
  for (int i = 0; i < P; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (P + 0.5));
    for (int it = 0; it < 100; ++it) {
      double Pn, dPn;
      legendre(P, x, Pn, dPn);
      double dx = Pn / dPn;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double Pn, dPn;
    legendre(P, x, Pn, dPn);
    o.xi[i] = x;
    o.w[i] = 2.0 / ((1.0 - x * x) * dPn * dPn);
  }
  // enforce exact symmetry of the rule
  for (int i = 0; i < P / 2; ++i) {
    double a = 0.5 * (o.xi[P - 1 - i] - o.xi[i]);
    o.xi[i] = -a; o.xi[P - 1 - i] = a;
    double w = 0.5 * (o.w[i] + o.w[P - 1 - i]);
    o.w[i] = o.w[P - 1 - i] = w;
  }
  if (P % 2) o.xi[P / 2] = 0.0;
  // barycentric differentiation matrix, diagonal from the zero row sum
  std::vector<double> lam(P, 1.0);
  for (int j = 0; j < P; ++j)
    for (int m = 0; m < P; ++m)
      if (m != j) lam[j] /= (o.xi[j] - o.xi[m]);
  o.D.assign(P * P, 0.0);
  for (int a = 0; a < P; ++a) {
    double s = 0.0;
    for (int b = 0; b < P; ++b) {
      if (a == b) continue;
      double v = (lam[b] / lam[a]) / (o.xi[a] - o.xi[b]);
      o.D[a * P + b] = v;
      s += v;
    }
    o.D[a * P + a] = -s;
  }
  o.lm.resize(P); o.lp.resize(P); o.gp.resize(P); o.gm.resize(P);
  for (int b = 0; b < P; ++b) {
    o.lm[b] = lagrange_1d(o.xi, b, -1.0);
    o.lp[b] = lagrange_1d(o.xi, b, 1.0);
  }
  for (int a = 0; a < P; ++a) {
    double P1, d1, P0, d0;
    legendre(p + 1, o.xi[a], P1, d1);
    legendre(p, o.xi[a], P0, d0);
    o.gp[a] = 0.5 * (d1 + d0);
    legendre(p + 1, -o.xi[a], P1, d1);
    legendre(p, -o.xi[a], P0, d0);
    o.gm[a] = 0.5 * (d1 + d0);
  }
  return o;
}

Geometry build_geometry(const MeshIn &m, const Ops1D &o) {
  const int d = m.dim, P = o.P;
  Geometry g;
  g.dim = d; g.P = P;
  g.Ns = (d == 2) ? P * P : P * P * P;
  g.Nfp = (d == 2) ? P : P * P;
  g.Nf = 2 * d * g.Nfp;
  g.n_elem = m.n_elem;
  const int Ns = g.Ns, Nf = g.Nf, nm = d * d + 1;
  GeoBasis bs = geo_basis(d, m.q, ref_solpts(d, o));
  GeoBasis bf = geo_basis(d, m.q, ref_fpts(d, o));
  const int nn = bs.nn;
  g.metric.assign((size_t)m.n_elem * nm * Ns, 0.0);
  g.J.assign((size_t)m.n_elem * Ns, 0.0);
  g.xsol.assign((size_t)m.n_elem * Ns * d, 0.0);
  g.xf.assign((size_t)m.n_elem * Nf * d, 0.0);
  g.Nvec.assign((size_t)m.n_elem * Nf * d, 0.0);
  std::atomic<int64_t> first_bad{-1};
  parallel_for(m.n_elem, [&](int64_t e) {
    double Xe[125 * 3];
    for (int n = 0; n < nn; ++n) {
      int64_t id = m.elem_nodes[e * nn + n];
      if (id < 0 || id >= m.n_node) throw FrError(FR_ERR_ARG, "element node id out of range");
      for (int j = 0; j < d; ++j) Xe[n * d + j] = m.node_xyz[id * d + j];
    }
    double x[3], A[9], adj[9];
    for (int i = 0; i < Ns; ++i) {
      map_point(d, bs, i, Xe, x, A);
      double J = adjugate(d, A, adj);
      if (!(J > 0.0)) { int64_t exp = -1; first_bad.compare_exchange_strong(exp, e); return; }
      for (int j = 0; j < d; ++j) g.xsol[((size_t)e * Ns + i) * d + j] = x[j];
      for (int kj = 0; kj < d * d; ++kj) g.metric[((size_t)e * nm + kj) * Ns + i] = adj[kj];
      g.metric[((size_t)e * nm + d * d) * Ns + i] = 1.0 / J;
      g.J[(size_t)e * Ns + i] = J;
    }
    for (int fp = 0; fp < Nf; ++fp) {
      map_point(d, bf, fp, Xe, x, A);
      double J = adjugate(d, A, adj);
      if (!(J > 0.0)) { int64_t exp = -1; first_bad.compare_exchange_strong(exp, e); return; }
      int f = fp / g.Nfp, k = f / 2;
      double s = (f % 2) ? 1.0 : -1.0;
      for (int j = 0; j < d; ++j) {
        g.xf[((size_t)e * Nf + fp) * d + j] = x[j];
        g.Nvec[((size_t)e * Nf + fp) * d + j] = s * adj[k * d + j];
      }
    }
  });
  if (first_bad.load() >= 0)
    throw FrError(FR_ERR_MESH, "element " + std::to_string(first_bad.load()) + " has a non-positive Jacobian");
  return g;
}

namespace {
struct Key {
  int64_t v[3];
  bool operator==(const Key &o) const { return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2]; }
};
struct KeyHash {
  size_t operator()(const Key &k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 3; ++i) { h ^= (uint64_t)k.v[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2); }
    return (size_t)h;
  }
};
}  // namespace

Connectivity build_connectivity(const MeshIn &m, const Ops1D &o, const Geometry &g) {
  const int d = m.dim, Nfp = g.Nfp, Nf = g.Nf, nface = 2 * d;
  const int64_t Ne = m.n_elem;
  Connectivity c;
  c.elem_mesh.assign(Ne, 0);
  for (int k = 0; k < m.n_mesh; ++k)
    for (int64_t e = m.mesh_begin[k]; e < m.mesh_begin[k + 1]; ++e) c.elem_mesh[e] = k;
  // domain scale
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t n = 0; n < m.n_node; ++n)
    for (int j = 0; j < d; ++j) {
      lo[j] = std::min(lo[j], m.node_xyz[n * d + j]);
      hi[j] = std::max(hi[j], m.node_xyz[n * d + j]);
    }
  double scale = 0.0;
  for (int j = 0; j < d; ++j) scale = std::max(scale, hi[j] - lo[j]);
  const double cell = 1e-6 * scale, tol = 1e-8 * scale;
  // face centroids (mean of the face's flux points)
  std::vector<double> cent((size_t)Ne * nface * 3, 0.0);
  for (int64_t e = 0; e < Ne; ++e)
    for (int f = 0; f < nface; ++f)
      for (int t = 0; t < Nfp; ++t)
        for (int j = 0; j < d; ++j)
          cent[((size_t)e * nface + f) * 3 + j] += g.xf[((size_t)e * Nf + f * Nfp + t) * d + j] / Nfp;
  auto quant = [&](const double *x) {
    Key k{{0, 0, 0}};
    for (int j = 0; j < d; ++j) k.v[j] = (int64_t)std::llround(x[j] / cell);
    return k;
  };
  std::unordered_map<Key, std::vector<int64_t>, KeyHash> grid;
  grid.reserve((size_t)Ne * d);
  for (int64_t e = 0; e < Ne; ++e)
    for (int f = 0; f < nface; ++f) {
      int32_t tag = m.face_bc[e * nface + f];
      if (tag != FR_FACE_AUTO && tag != FR_BC_WALL && tag != FR_BC_FARFIELD && !(m.allow_mortar && tag == BC_MORTAR))
        throw FrError(FR_ERR_ARG, "unknown face tag");
      if (tag == FR_FACE_AUTO) grid[quant(&cent[((size_t)e * nface + f) * 3])].push_back(e * nface + f);
    }
  std::vector<double> shifts(3, 0.0);
  for (int k = 0; k < m.n_periodic; ++k)
    for (int sg = 1; sg >= -1; sg -= 2)
      for (int j = 0; j < 3; ++j) shifts.push_back(j < d ? sg * m.periodic_vec[k * d + j] : 0.0);
  const int nshift = (int)shifts.size() / 3;
  std::vector<int64_t> partner((size_t)Ne * nface, -1);
  std::vector<int> partner_shift((size_t)Ne * nface, -1);
  for (int64_t a = 0; a < Ne * nface; ++a) {
    int64_t e = a / nface;
    int f = (int)(a % nface);
    if (m.face_bc[e * nface + f] != FR_FACE_AUTO || partner[a] >= 0) continue;
    const double *ca = &cent[(size_t)a * 3];
    int64_t found = -1;
    int fs = -1;
    for (int s = 0; s < nshift && found < 0; ++s) {
      double tgt[3];
      for (int j = 0; j < 3; ++j) tgt[j] = ca[j] + shifts[s * 3 + j];
      Key k0 = quant(tgt);
      int nb = (d == 2) ? 9 : 27;
      for (int q = 0; q < nb && found < 0; ++q) {
        Key k = k0;
        k.v[0] += q % 3 - 1;
        k.v[1] += (q / 3) % 3 - 1;
        if (d == 3) k.v[2] += q / 9 - 1;
        auto it = grid.find(k);
        if (it == grid.end()) continue;
        for (int64_t b : it->second) {
          // faces of different meshes of a batch are never paired, even where they coincide
          if (b == a || partner[b] >= 0 || c.elem_mesh[b / nface] != c.elem_mesh[e]) continue;
          const double *cb = &cent[(size_t)b * 3];
          double dist = 0.0;
          for (int j = 0; j < d; ++j) dist = std::max(dist, std::fabs(cb[j] - tgt[j]));
          if (dist < tol) { found = b; fs = s; break; }
        }
      }
    }
    if (found < 0)
      throw FrError(FR_ERR_MESH, "unmatched face: element " + std::to_string(e) + " face " + std::to_string(f));
    partner[a] = found;
    partner[found] = a;
    partner_shift[a] = fs;
    partner_shift[found] = fs == 0 ? 0 : (fs % 2 ? fs + 1 : fs - 1);  // opposite translation
  }
  // flux-point pairs, L = the smaller (element, face)
  for (int64_t a = 0; a < Ne * nface; ++a) {
    int64_t b = partner[a];
    if (b < 0 || b < a) continue;
    int64_t e = a / nface, e2 = b / nface;
    int f = (int)(a % nface), f2 = (int)(b % nface);
    const double *sh = &shifts[partner_shift[a] * 3];
    std::vector<int> used(Nfp, 0);
    for (int t = 0; t < Nfp; ++t) {
      const double *xa = &g.xf[((size_t)e * Nf + f * Nfp + t) * d];
      int best = -1;
      double bd = 1e300;
      for (int t2 = 0; t2 < Nfp; ++t2) {
        const double *xb = &g.xf[((size_t)e2 * Nf + f2 * Nfp + t2) * d];
        double dist = 0.0;
        for (int j = 0; j < d; ++j) dist += (xa[j] + sh[j] - xb[j]) * (xa[j] + sh[j] - xb[j]);
        if (dist < bd) { bd = dist; best = t2; }
      }
      if (std::sqrt(bd) > 1e-7 * scale || used[best])
        throw FrError(FR_ERR_MESH, "non-conforming face pair at element " + std::to_string(e));
      used[best] = 1;
      int fpL = f * Nfp + t, fpR = f2 * Nfp + best;
      c.pairL.push_back((int32_t)(e * Nf + fpL));
      c.pairR.push_back((int32_t)(e2 * Nf + fpR));
      const double *N = &g.Nvec[((size_t)e * Nf + fpL) * d];
      double mag = 0.0;
      for (int j = 0; j < d; ++j) mag += N[j] * N[j];
      mag = std::sqrt(mag);
      for (int j = 0; j < d; ++j) c.pair_nrm.push_back(N[j] / mag);
      c.pair_nrm.push_back(mag);
    }
  }
  // boundary flux points: walls, then far field, then (degree-group solvers) mortar points
  for (int pass = 0; pass < 3; ++pass) {
    int want = pass == 0 ? FR_BC_WALL : (pass == 1 ? FR_BC_FARFIELD : BC_MORTAR);
    if (pass == 2) c.n_bc = (int64_t)c.bnd.size();
    if (pass == 0) c.wall_mesh_begin.assign(m.n_mesh + 1, 0);
    for (int64_t e = 0; e < Ne; ++e)
      for (int f = 0; f < nface; ++f) {
        if (m.face_bc[e * nface + f] != want) continue;
        for (int t = 0; t < Nfp; ++t) {
          int fp = f * Nfp + t;
          c.bnd.push_back((int32_t)(e * Nf + fp));
          const double *N = &g.Nvec[((size_t)e * Nf + fp) * d];
          double mag = 0.0;
          for (int j = 0; j < d; ++j) mag += N[j] * N[j];
          mag = std::sqrt(mag);
          for (int j = 0; j < d; ++j) c.bnd_nrm.push_back(N[j] / mag);
          c.bnd_nrm.push_back(mag);
          double w = (d == 2) ? o.w[t] : o.w[t % o.P] * o.w[t / o.P];
          c.bnd_w.push_back(w);
          if (pass == 0) c.wall_mesh_begin[c.elem_mesh[e] + 1]++;
        }
      }
    if (pass == 0) {
      c.n_wall = (int64_t)c.bnd.size();
      for (int k = 0; k < m.n_mesh; ++k) c.wall_mesh_begin[k + 1] += c.wall_mesh_begin[k];
    }
  }
  if ((int64_t)Ne * Nf >= ((int64_t)1 << 30))
    throw FrError(FR_ERR_ARG, "mesh too large for 30-bit flux-point codes");
  // element-side view of the same connectivity
  c.nbr.assign((size_t)Ne * Nf, INT32_MIN);
  c.fnrm.assign((size_t)Ne * (d + 1) * Nf, 0.0);
  for (size_t q = 0; q < c.pairL.size(); ++q) {
    const int32_t L = c.pairL[q], R = c.pairR[q];
    c.nbr[L] = R;
    c.nbr[R] = L | NBR_R_BIT;
    const int64_t eL = L / Nf, eR = R / Nf;
    const int fL = L % Nf, fR = R % Nf;
    for (int j = 0; j <= d; ++j) {
      const double nj = c.pair_nrm[q * (d + 1) + j];
      c.fnrm[((size_t)eL * (d + 1) + j) * Nf + fL] = nj;
      c.fnrm[((size_t)eR * (d + 1) + j) * Nf + fR] = j < d ? -nj : nj;  // |N| of the pair on both sides
    }
  }
  for (size_t b = 0; b < c.bnd.size(); ++b) {
    const int32_t C = c.bnd[b];
    c.nbr[C] = -(int32_t)b - 1;
    const int64_t e = C / Nf;
    const int fp = C % Nf;
    for (int j = 0; j <= d; ++j) c.fnrm[((size_t)e * (d + 1) + j) * Nf + fp] = c.bnd_nrm[b * (d + 1) + j];
  }
  for (size_t k = 0; k < c.nbr.size(); ++k)
    if (c.nbr[k] == INT32_MIN) throw FrError(FR_ERR_MESH, "flux point without a partner or boundary tag");
  return c;
}

Probe locate_probe(const MeshIn &m, const Ops1D &o, const double *xp, int mesh) {
  const int d = m.dim;
  std::vector<double> nodes = gll_nodes(m.q);
  const int Q = m.q + 1;
  int nn = 1;
  for (int k = 0; k < d; ++k) nn *= Q;
  int64_t e0 = m.mesh_begin[mesh], e1 = m.mesh_begin[mesh + 1];
  for (int64_t e = e0; e < e1; ++e) {
    double Xe[125 * 3];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int n = 0; n < nn; ++n) {
      int64_t id = m.elem_nodes[e * nn + n];
      for (int j = 0; j < d; ++j) {
        Xe[n * d + j] = m.node_xyz[id * d + j];
        lo[j] = std::min(lo[j], Xe[n * d + j]);
        hi[j] = std::max(hi[j], Xe[n * d + j]);
      }
    }
    double span = 0.0;
    for (int j = 0; j < d; ++j) span = std::max(span, hi[j] - lo[j]);
    bool near = true;
    for (int j = 0; j < d; ++j) near = near && xp[j] >= lo[j] - 0.25 * span && xp[j] <= hi[j] + 0.25 * span;
    if (!near) continue;
    double xi[3] = {0.0, 0.0, 0.0};
    bool ok = false;
    int polish = 0;
    for (int it = 0; it < 60; ++it) {
      std::vector<double> ref(xi, xi + d);
      GeoBasis b = geo_basis(d, m.q, ref);
      double x[3], A[9], adj[9];
      map_point(d, b, 0, Xe, x, A);
      double J = adjugate(d, A, adj);
      if (J == 0.0) break;
      double r[3], dxi[3];
      for (int j = 0; j < d; ++j) r[j] = x[j] - xp[j];
      double mx = 0.0, mxi = 0.0;
      for (int k = 0; k < d; ++k) {
        dxi[k] = 0.0;
        for (int j = 0; j < d; ++j) dxi[k] += adj[k * d + j] * r[j] / J;
        xi[k] -= dxi[k];
        mx = std::max(mx, std::fabs(dxi[k]));
        mxi = std::max(mxi, std::fabs(xi[k]));
      }
      if (mxi > 3.0) break;
      // converged to 1e-12 in reference coordinates, then two polishing iterations (round-off in x
      // limits |dxi| to ~eps |x| / h, above 1e-14 for small elements far from the origin)
      if (ok) {
        if (++polish == 2) break;
      } else if (mx < 1e-12) {
        ok = true;
      }
    }
    double mxi = 0.0;
    for (int k = 0; k < d; ++k) mxi = std::max(mxi, std::fabs(xi[k]));
    if (ok && mxi <= 1.0 + 1e-12) {
      Probe pr;
      pr.elem = e;
      pr.mesh = mesh;
      pr.xi.assign(xi, xi + d);
      int P = o.P, Ns = (d == 2) ? P * P : P * P * P;
      pr.weights.assign(Ns, 1.0);
      pr.dweights.assign((size_t)d * Ns, 1.0);
      for (int i = 0; i < Ns; ++i) {
        int ii[3] = {i % P, (i / P) % P, i / (P * P)};
        for (int k = 0; k < d; ++k) {
          const double l = lagrange_1d(o.xi, ii[k], xi[k]), dl = lagrange_1d_deriv(o.xi, ii[k], xi[k]);
          pr.weights[i] *= l;
          for (int kd = 0; kd < d; ++kd) pr.dweights[(size_t)kd * Ns + i] *= (kd == k ? dl : l);
        }
      }
      // d xi / d X_n = -A^{-1} phi_n(xi) at the located point
      std::vector<double> ref(xi, xi + d);
      GeoBasis b = geo_basis(d, m.q, ref);
      double x[3], A[9], adj[9];
      map_point(d, b, 0, Xe, x, A);
      const double J = adjugate(d, A, adj);
      pr.dxi.assign((size_t)nn * d * d, 0.0);
      pr.nodes.resize(nn);
      for (int n = 0; n < nn; ++n) {
        pr.nodes[n] = m.elem_nodes[e * nn + n];
        for (int j = 0; j < d; ++j)
          for (int k = 0; k < d; ++k) pr.dxi[((size_t)n * d + j) * d + k] = -adj[k * d + j] / J * b.phi[n];
      }
      return pr;
    }
  }
  throw FrError(FR_ERR_MESH, "probe is outside every element of its mesh");
}

std::vector<double> ref_flux_points(int dim, const Ops1D &o) { return ref_fpts(dim, o); }

std::vector<double> map_ref_points(const MeshIn &m, int64_t e, const std::vector<double> &ref) {
  const int d = m.dim;
  GeoBasis b = geo_basis(d, m.q, ref);
  std::vector<double> Xe((size_t)b.nn * d);
  for (int n = 0; n < b.nn; ++n)
    for (int j = 0; j < d; ++j) Xe[(size_t)n * d + j] = m.node_xyz[m.elem_nodes[e * b.nn + n] * d + j];
  std::vector<double> x((size_t)b.npts * d);
  for (int a = 0; a < b.npts; ++a) {
    double A[9];
    map_point(d, b, a, Xe.data(), &x[(size_t)a * d], A);
  }
  return x;
}

GeoAdj build_geo_adj(const MeshIn &m, const Ops1D &o) {
  const int d = m.dim, Q = m.q + 1;
  int nn = 1;
  for (int k = 0; k < d; ++k) nn *= Q;
  GeoAdj g;
  g.nn = nn;
  GeoBasis bs = geo_basis(d, m.q, ref_solpts(d, o));
  GeoBasis bf = geo_basis(d, m.q, ref_fpts(d, o));
  g.dphi_s = bs.dphi;
  g.dphi_f = bf.dphi;
  g.Xe.resize((size_t)m.n_elem * nn * d);
  std::vector<int32_t> cnt(m.n_node + 1, 0);
  for (int64_t e = 0; e < m.n_elem; ++e)
    for (int n = 0; n < nn; ++n) {
      const int64_t id = m.elem_nodes[e * nn + n];
      if (id < 0 || id >= m.n_node) throw FrError(FR_ERR_MESH, "element node id out of range");
      for (int j = 0; j < d; ++j) g.Xe[((size_t)e * nn + n) * d + j] = m.node_xyz[id * d + j];
      cnt[id + 1]++;
    }
  if ((int64_t)m.n_elem * nn >= ((int64_t)1 << 31)) throw FrError(FR_ERR_ARG, "mesh too large for the node incidence");
  for (int64_t i = 0; i < m.n_node; ++i) cnt[i + 1] += cnt[i];
  g.inc_ptr = cnt;
  g.inc.resize((size_t)m.n_elem * nn);
  std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < m.n_elem; ++e)
    for (int n = 0; n < nn; ++n) g.inc[pos[m.elem_nodes[e * nn + n]]++] = (int32_t)(e * nn + n);
  return g;
}

}  // namespace frmi
