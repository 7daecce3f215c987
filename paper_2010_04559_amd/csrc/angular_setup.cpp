// Host-side angular discretisation (see angular_setup.h).
#include "angular_setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace tr {

namespace {

constexpr double kPi = 3.14159265358979323846;

V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }
V3 unit(V3 a) { return scale(a, 1.0 / norm(a)); }

V3 octant_sign(int o) { return {(o & 1) ? -1.0 : 1.0, (o & 2) ? -1.0 : 1.0, (o & 4) ? -1.0 : 1.0}; }

// central projection onto the octahedron face s . x = 1
V3 project(V3 a, V3 s) { return scale(a, 1.0 / dot(a, s)); }

double safe_acos(double c) { return std::acos(std::min(1.0, std::max(-1.0, c))); }

void split(std::vector<PatchNode> &t, int i) {
  PatchNode p = t[i];
  V3 a = p.v[0], b = p.v[1], c = p.v[2];
  V3 mab = unit(add(a, b)), mbc = unit(add(b, c)), mca = unit(add(c, a));
  V3 kids[4][3] = {{a, mab, mca}, {mab, b, mbc}, {mca, mbc, c}, {mab, mbc, mca}};
  for (int k = 0; k < 4; ++k) {
    PatchNode ch;
    for (int e = 0; e < 3; ++e) ch.v[e] = kids[k][e];
    ch.level = p.level + 1;
    ch.octant = p.octant;
    ch.parent = i;
    t.push_back(ch);
    t[i].child[k] = (int)t.size() - 1;
  }
}

int required_level(const RefineSpec &s, const PatchNode &p) {
  if (s.band_lmax > 0) {
    // Section 5.5: bands of the largest vertex Omega_z, strict thresholds
    double z = p.v[0].z;
    for (int e = 1; e < 3; ++e) z = std::max(z, p.v[e].z);
    const int lev = z > 0.97 ? s.band_lmax : z > 0.9 ? s.band_lmax - 1 : z > 0.8 ? s.band_lmax - 2
                  : z > 0.6 ? s.band_lmax - 3 : s.band_lmax - 4;
    return std::max(lev, 0);
  }
  if (s.cone_extra_levels <= 0) return s.base_level;
  V3 ax = unit(s.cone_axis);
  double c = std::cos(s.cone_half_angle_deg * kPi / 180.0);
  for (int e = 0; e < 3; ++e)
    if (dot(p.v[e], ax) > c) return s.base_level + s.cone_extra_levels;
  return s.base_level;
}

void collect(const std::vector<PatchNode> &t, int i, int cut, std::vector<int> &out) {
  const PatchNode &p = t[i];
  if (p.leaf() || p.level == cut) {
    out.push_back(i);
    return;
  }
  for (int k = 0; k < 4; ++k) collect(t, p.child[k], cut, out);
}

std::vector<int> leaves(const std::vector<PatchNode> &t, int cut) {
  std::vector<int> out;
  for (int r = 0; r < 8; ++r) collect(t, r, cut, out);
  return out;
}

void apply_rule(std::vector<PatchNode> &t, const RefineSpec &s) {
  std::vector<int> stack = leaves(t, 1 << 30);
  while (!stack.empty()) {
    int i = stack.back();
    stack.pop_back();
    if (t[i].level < required_level(s, t[i])) {
      split(t, i);
      for (int k = 0; k < 4; ++k) stack.push_back(t[i].child[k]);
    }
  }
}

// Leaves sharing a boundary segment: the midpoint of an edge of one lies
// strictly inside an edge (great-circle arc) of the other.
bool neighbours(const PatchNode &a, const PatchNode &b) {
  for (int e = 0; e < 3; ++e) {
    V3 m = unit(add(a.v[e], a.v[(e + 1) % 3]));
    for (int f = 0; f < 3; ++f) {
      V3 u = b.v[f], v = b.v[(f + 1) % 3];
      double um = safe_acos(dot(u, m)), mv = safe_acos(dot(m, v)), uv = safe_acos(dot(u, v));
      if (um > 1e-12 && mv > 1e-12 && std::fabs(um + mv - uv) < 1e-12) return true;
    }
  }
  return false;
}

// ---------------------------------------------------------------- Gauss
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  // Newton iteration on P_n from the Chebyshev-like initial guess
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
      double p2 = p1;
      p1 = p0;
      p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    dp = n * (z * p0 - p1) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

double patch_angle(const PatchNode &p) {
  double m = 0;
  for (int e = 0; e < 3; ++e) m = std::max(m, safe_acos(dot(p.v[e], p.v[(e + 1) % 3])));
  return m;
}

// Accurate rule on a patch: the flat (projected) triangle is cut into three
// quadrilaterals at its centroid and edge midpoints; each gets a tensor
// Gauss-Legendre rule through its bilinear map; the gnomonic Jacobian
// dOmega = dA / (sqrt(3) |x|^3) maps the result to the sphere.
void accurate_rule(const PatchNode &p, int order, std::vector<V3> &pts, std::vector<double> &wts) {
  V3 s = octant_sign(p.octant);
  V3 f[3] = {project(p.v[0], s), project(p.v[1], s), project(p.v[2], s)};
  V3 g = scale(add(add(f[0], f[1]), f[2]), 1.0 / 3.0);
  V3 m01 = scale(add(f[0], f[1]), 0.5), m12 = scale(add(f[1], f[2]), 0.5), m20 = scale(add(f[2], f[0]), 0.5);
  V3 quads[3][4] = {{f[0], m01, g, m20}, {f[1], m12, g, m01}, {f[2], m20, g, m12}};
  double th = patch_angle(p);
  int n = (int)std::ceil(8.0 + 6.0 * th + 0.9 * order * th);
  n = std::max(10, std::min(n, 72));
  std::vector<double> gx, gw;
  gauss_legendre(n, gx, gw);
  pts.clear();
  wts.clear();
  const double inv_sqrt3 = 1.0 / std::sqrt(3.0);
  for (int q = 0; q < 3; ++q) {
    const V3 *Q = quads[q];
    for (int a = 0; a < n; ++a) {
      double u = 0.5 * (gx[a] + 1.0), wu = 0.5 * gw[a];
      for (int b = 0; b < n; ++b) {
        double v = 0.5 * (gx[b] + 1.0), wv = 0.5 * gw[b];
        V3 x = add(add(scale(Q[0], (1 - u) * (1 - v)), scale(Q[1], u * (1 - v))),
                   add(scale(Q[2], u * v), scale(Q[3], (1 - u) * v)));
        V3 du = add(scale(sub(Q[1], Q[0]), 1 - v), scale(sub(Q[2], Q[3]), v));
        V3 dv = add(scale(sub(Q[3], Q[0]), 1 - u), scale(sub(Q[2], Q[1]), u));
        double jac = norm(cross(du, dv));
        double r = norm(x);
        pts.push_back(scale(x, 1.0 / r));
        wts.push_back(wu * wv * jac * inv_sqrt3 / (r * r * r));
      }
    }
  }
}

// Orthonormal real spherical harmonics Y_{n,o}, index n*n + n + o.
void real_harmonics(int L, const V3 &om, double *Y) {
  const double x = std::max(-1.0, std::min(1.0, om.z));
  const double sn = std::sqrt(std::max(0.0, 1.0 - x * x));
  const double phi = std::atan2(om.y, om.x);
  std::vector<double> P((L + 1) * (L + 1), 0.0);  // P[n*(L+1)+m]
  double pmm = 1.0 / std::sqrt(4.0 * kPi);
  for (int m = 0; m <= L; ++m) {
    if (m > 0) pmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * sn;
    P[m * (L + 1) + m] = pmm;
    if (m < L) P[(m + 1) * (L + 1) + m] = std::sqrt(2.0 * m + 3.0) * x * pmm;
    for (int n = m + 2; n <= L; ++n) {
      double a = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      double b = std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
      P[n * (L + 1) + m] = a * (x * P[(n - 1) * (L + 1) + m] - b * P[(n - 2) * (L + 1) + m]);
    }
  }
  const double r2 = std::sqrt(2.0);
  for (int n = 0; n <= L; ++n) {
    Y[n * n + n] = P[n * (L + 1)];
    for (int m = 1; m <= n; ++m) {
      Y[n * n + n + m] = r2 * P[n * (L + 1) + m] * std::cos(m * phi);
      Y[n * n + n - m] = r2 * P[n * (L + 1) + m] * std::sin(m * phi);
    }
  }
}

}  // namespace

double spherical_area(const PatchNode &p) {
  double num = std::fabs(dot(p.v[0], cross(p.v[1], p.v[2])));
  double den = 1.0 + dot(p.v[0], p.v[1]) + dot(p.v[1], p.v[2]) + dot(p.v[2], p.v[0]);
  return 2.0 * std::atan2(num, den);
}

void lin_basis(const PatchNode &p, const V3 &om, double psi[3]) {
  V3 s = octant_sign(p.octant);
  V3 f0 = project(p.v[0], s), f1 = project(p.v[1], s), f2 = project(p.v[2], s);
  V3 x = project(om, s);
  // barycentric coordinates by Cramer's rule on [f0 f1 f2] lambda = x
  double det = dot(f0, cross(f1, f2));
  psi[0] = dot(x, cross(f1, f2)) / det;
  psi[1] = dot(f0, cross(x, f2)) / det;
  psi[2] = dot(f0, cross(f1, x)) / det;
}

void patch_x_integrals(const PatchNode &p, int order, std::vector<double> &X, bool const_basis) {
  const int K = (order + 1) * (order + 1);
  X.assign(3 * K, 0.0);
  std::vector<V3> pts;
  std::vector<double> wts;
  accurate_rule(p, order, pts, wts);
  std::vector<double> Y(K);
  for (size_t t = 0; t < pts.size(); ++t) {
    double psi[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};
    if (!const_basis) lin_basis(p, pts[t], psi);
    real_harmonics(order, pts[t], Y.data());
    for (int m = 0; m < 3; ++m) {
      double c = wts[t] * psi[m];
      double *row = &X[m * K];
      for (int k = 0; k < K; ++k) row[k] += c * Y[k];
    }
  }
}

void scatter_matrix(const HostAngular &ang, int level, const std::vector<double> &moments,
                    std::vector<double> &St, std::vector<double> *Xout) {
  const HostLevel &L = ang.lv[level];
  const int order = (int)moments.size() - 1;
  const int K = (order + 1) * (order + 1);
  std::vector<double> X((size_t)L.A * K);
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < L.P; ++q) {
    std::vector<double> Xq;
    patch_x_integrals(ang.tree[L.node[q]], order, Xq, ang.const_basis);
    std::copy(Xq.begin(), Xq.end(), X.begin() + (size_t)3 * q * K);
  }
  std::vector<double> F(K);
  for (int n = 0; n <= order; ++n)
    for (int o = -n; o <= n; ++o) F[n * n + n + o] = moments[n];
  if (Xout) *Xout = X;
  St.assign((size_t)L.A * L.A, 0.0);
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < L.A; ++a) {
    const double *xa = &X[(size_t)a * K];
    for (int b = 0; b <= a; ++b) {
      const double *xb = &X[(size_t)b * K];
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += xa[k] * F[k] * xb[k];
      St[(size_t)a * L.A + b] = acc;
      St[(size_t)b * L.A + a] = acc;
    }
  }
}

bool build_angular(const RefineSpec &spec, HostAngular &out, std::string &err) {
  if (spec.base_level < 0 || spec.base_level > 6 || spec.cone_extra_levels < 0 ||
      spec.base_level + spec.cone_extra_levels > 8) {
    err = "angular refinement levels out of range (base 0..6, base+extra <= 8)";
    return false;
  }
  if (spec.band_lmax < 0 || spec.band_lmax > 8 || (spec.band_lmax > 0 && spec.cone_extra_levels > 0)) {
    err = "z-band refinement: band_lmax in 0..8 (0 = off), not together with a cone";
    return false;
  }
  std::vector<PatchNode> &t = out.tree;
  t.clear();
  for (int o = 0; o < 8; ++o) {
    PatchNode r;
    V3 s = octant_sign(o);
    r.v[0] = {s.x, 0, 0};
    r.v[1] = {0, s.y, 0};
    r.v[2] = {0, 0, s.z};
    r.octant = o;
    t.push_back(r);
  }
  apply_rule(t, spec);
  if (spec.closure && spec.cone_extra_levels > 0) {
    for (int guard = 0; guard < 64; ++guard) {
      std::vector<int> lv = leaves(t, 1 << 30);
      std::vector<char> todo(lv.size(), 0);
      bool any = false;
      for (size_t i = 0; i < lv.size(); ++i)
        for (size_t j = i + 1; j < lv.size(); ++j) {
          int li = t[lv[i]].level, lj = t[lv[j]].level;
          if (std::abs(li - lj) <= 2) continue;
          if (!neighbours(t[lv[i]], t[lv[j]]) && !neighbours(t[lv[j]], t[lv[i]])) continue;
          todo[li < lj ? i : j] = 1;
          any = true;
        }
      if (!any) break;
      for (size_t i = 0; i < lv.size(); ++i)
        if (todo[i]) split(t, lv[i]);
      apply_rule(t, spec);
    }
  }
  int maxlev = 0;
  for (int i : leaves(t, 1 << 30)) maxlev = std::max(maxlev, t[i].level);
  out.lv.assign(maxlev + 1, HostLevel());
  out.const_basis = spec.const_basis;

  const double Psi[3][3] = {{4.0 / 6, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 4.0 / 6, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 4.0 / 6}};
  for (int l = 0; l <= maxlev; ++l) {
    HostLevel &L = out.lv[l];
    L.node = leaves(t, l);
    L.P = (int)L.node.size();
    L.A = 3 * L.P;
    L.octant.resize(L.P);
    L.omega.assign((size_t)L.A * 3, 0.0);
    L.w.assign(L.A, 0.0);
    L.ipsi.assign(L.A, 0.0);
    L.iom.assign((size_t)L.A * 3, 0.0);
    for (int q = 0; q < L.P; ++q) {
      const PatchNode &p = t[L.node[q]];
      L.octant[q] = p.octant;
      V3 s = octant_sign(p.octant);
      V3 f[3] = {project(p.v[0], s), project(p.v[1], s), project(p.v[2], s)};
      // exact integrals of the Lin functions
      std::vector<V3> pts;
      std::vector<double> wts;
      accurate_rule(p, 0, pts, wts);
      double ip[3] = {0, 0, 0};
      for (size_t k = 0; k < pts.size(); ++k) {
        double ps[3];
        lin_basis(p, pts[k], ps);
        for (int m = 0; m < 3; ++m) ip[m] += wts[k] * ps[m];
      }
      double sum_ip = ip[0] + ip[1] + ip[2];
      if (spec.const_basis) {
        // Const: three coincident ordinates at the mean direction
        // int_q Omega / |q| (not a unit vector), a third of |q| each
        V3 mo{0, 0, 0};
        double area = 0;
        for (size_t k = 0; k < pts.size(); ++k) {
          mo = add(mo, scale(pts[k], wts[k]));
          area += wts[k];
        }
        const V3 om = scale(mo, 1.0 / area);
        for (int k = 0; k < 3; ++k) {
          L.ipsi[3 * q + k] = area / 3.0;
          L.omega[3 * (3 * q + k) + 0] = om.x;
          L.omega[3 * (3 * q + k) + 1] = om.y;
          L.omega[3 * (3 * q + k) + 2] = om.z;
          L.w[3 * q + k] = area / 3.0;
        }
      } else {
        for (int m = 0; m < 3; ++m) L.ipsi[3 * q + m] = ip[m];
        // 3-point rule: barycentric (2/3, 1/6, 1/6); psi_d(Omega_k) = Psi[k][d];
        // weights w = Psi^{-1} int psi (Psi^{-1} = 2 I - J / 3)
        for (int k = 0; k < 3; ++k) {
          V3 x = add(add(scale(f[0], Psi[k][0]), scale(f[1], Psi[k][1])), scale(f[2], Psi[k][2]));
          V3 om = unit(x);
          L.omega[3 * (3 * q + k) + 0] = om.x;
          L.omega[3 * (3 * q + k) + 1] = om.y;
          L.omega[3 * (3 * q + k) + 2] = om.z;
          L.w[3 * q + k] = 2.0 * ip[k] - sum_ip / 3.0;
        }
      }
      for (int m = 0; m < 3; ++m)
        for (int xi = 0; xi < 3; ++xi) {
          double acc = 0;
          for (int k = 0; k < 3; ++k) acc += Psi[k][m] * L.w[3 * q + k] * L.omega[3 * (3 * q + k) + xi];
          L.iom[3 * (3 * q + m) + xi] = acc;
        }
    }
    if (l > 0) {
      const HostLevel &Cl = out.lv[l - 1];
      L.owner.assign(L.P, -1);
      L.pblk.assign((size_t)L.P * 9, 0.0);
      L.first_child.assign(Cl.P, -1);
      L.n_child.assign(Cl.P, 0);
      int c = 0;
      for (int p = 0; p < Cl.P; ++p) {
        int nd = Cl.node[p];
        L.first_child[p] = c;
        if (t[nd].leaf() || t[nd].level < l - 1) {
          // unrefined on this level: the same patch
          L.owner[c] = p;
          for (int k = 0; k < 3; ++k) L.pblk[(size_t)c * 9 + k * 3 + k] = 1.0;
          L.n_child[p] = 1;
          ++c;
        } else {
          for (int k = 0; k < 4; ++k, ++c) {
            if (L.node[c] != t[nd].child[k]) {
              err = "internal: child order mismatch";
              return false;
            }
            L.owner[c] = p;
            for (int e = 0; e < 3; ++e) {
              double ps[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};  // Const: the parent's value
              if (!spec.const_basis) lin_basis(t[nd], t[L.node[c]].v[e], ps);
              for (int d = 0; d < 3; ++d) L.pblk[(size_t)c * 9 + e * 3 + d] = ps[d];
            }
          }
          L.n_child[p] = 4;
        }
      }
      if (c != L.P) {
        err = "internal: level nesting mismatch";
        return false;
      }
    }
  }
  return true;
}

}  // namespace tr
