// Height-function quadrature on boxes cut by quadric or polynomial level sets
// (see quadrature.hpp).
#include "quadrature.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>
#include <stdexcept>

namespace cc {

static const double kNaN = std::numeric_limits<double>::quiet_NaN();

double Quadric::eval(const double* x) const {
  double v = c;
  for (int i = 0; i < e; ++i) {
    v += b[i] * x[i];
    double t = 0.0;
    for (int j = 0; j < e; ++j) t += Q[i][j] * x[j];
    v += x[i] * t;
  }
  return v;
}

void Quadric::grad(const double* x, double* g) const {
  for (int i = 0; i < e; ++i) {
    double t = 0.0;
    for (int j = 0; j < e; ++j) t += Q[i][j] * x[j];
    g[i] = 2.0 * t + b[i];
  }
}

Quadric Quadric::restrict_to(int k, double val) const {
  Quadric r;
  r.e = e - 1;
  int map[3], m = 0;
  for (int i = 0; i < e; ++i)
    if (i != k) map[m++] = i;
  for (int i = 0; i < r.e; ++i) {
    for (int j = 0; j < r.e; ++j) r.Q[i][j] = Q[map[i]][map[j]];
    r.b[i] = b[map[i]] + 2.0 * Q[k][map[i]] * val;
  }
  r.c = c + b[k] * val + Q[k][k] * val * val;
  return r;
}

Quadric ellipsoid_quadric(const double center[3], const double axes[3], const double rot[9]) {
  // A = R diag(1/a^2) R^T; phi = (x - c)^T A (x - c) - 1
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int t = 0; t < 3; ++t) s += rot[3 * i + t] * rot[3 * j + t] / (axes[t] * axes[t]);
      A[i][j] = s;
    }
  Quadric q;
  q.e = 3;
  double ctac = 0.0;
  for (int i = 0; i < 3; ++i) {
    double Ac = 0.0;
    for (int j = 0; j < 3; ++j) {
      q.Q[i][j] = A[i][j];
      Ac += A[i][j] * center[j];
    }
    q.b[i] = -2.0 * Ac;
    ctac += center[i] * Ac;
  }
  q.c = ctac - 1.0;
  return q;
}

// ------------------------------------------------------------ polynomials
namespace {

inline int pstride(int e, int i) { return e == 3 ? (i == 0 ? 25 : (i == 1 ? 5 : 1)) : (e == 2 ? (i == 0 ? 5 : 1) : 1); }

// calls fn(a, index) for every exponent a (a[i] = 0 for i >= e) of total degree <= 4
template <class Fn>
void for_each_exp(int e, Fn fn) {
  int a[3] = {0, 0, 0};
  const int m0 = e > 0 ? Poly::kDeg : 0;
  for (a[0] = 0; a[0] <= m0; ++a[0]) {
    const int m1 = e > 1 ? Poly::kDeg - a[0] : 0;
    for (a[1] = 0; a[1] <= m1; ++a[1]) {
      const int m2 = e > 2 ? Poly::kDeg - a[0] - a[1] : 0;
      for (a[2] = 0; a[2] <= m2; ++a[2]) {
        int id = 0;
        for (int i = 0; i < e; ++i) id += a[i] * pstride(e, i);
        fn(a, id);
      }
    }
  }
}

void powers(int e, const double* x, double pw[3][5]) {
  for (int i = 0; i < e; ++i) {
    pw[i][0] = 1.0;
    for (int j = 1; j <= Poly::kDeg; ++j) pw[i][j] = pw[i][j - 1] * x[i];
  }
}

Poly poly_const(int e, double v) {
  Poly p;
  p.e = e;
  p.c[0] = v;
  return p;
}

// x_i - shift in 3 variables
Poly poly_coord(int i, double shift) {
  Poly p;
  p.e = 3;
  p.c[0] = -shift;
  p.c[pstride(3, i)] = 1.0;
  return p;
}

Poly poly_axpy(double a, const Poly& x, const Poly& y) {  // a x + y
  Poly r = y;
  for (int t = 0; t < 125; ++t) r.c[t] += a * x.c[t];
  return r;
}

Poly poly_mul(const Poly& x, const Poly& y) {
  Poly r;
  r.e = x.e;
  for_each_exp(x.e, [&](const int* a, int ia) {
    if (x.c[ia] == 0.0) return;
    for_each_exp(x.e, [&](const int* b, int ib) {
      if (y.c[ib] == 0.0) return;
      int deg = 0, id = 0;
      for (int i = 0; i < x.e; ++i) {
        deg += a[i] + b[i];
        id += (a[i] + b[i]) * pstride(x.e, i);
      }
      if (deg > Poly::kDeg) throw std::runtime_error("polynomial level set above degree 4");
      r.c[id] += x.c[ia] * y.c[ib];
    });
  });
  return r;
}

double horner(const double* a, int deg, double t) {
  double v = a[deg];
  for (int j = deg - 1; j >= 0; --j) v = v * t + a[j];
  return v;
}

}  // namespace

double Poly::eval(const double* x) const {
  double pw[3][5];
  powers(e, x, pw);
  double v = 0.0;
  for_each_exp(e, [&](const int* a, int id) {
    if (c[id] == 0.0) return;
    double t = c[id];
    for (int i = 0; i < e; ++i) t *= pw[i][a[i]];
    v += t;
  });
  return v;
}

void Poly::grad(const double* x, double* g) const {
  double pw[3][5];
  powers(e, x, pw);
  for (int k = 0; k < e; ++k) g[k] = 0.0;
  for_each_exp(e, [&](const int* a, int id) {
    if (c[id] == 0.0) return;
    for (int k = 0; k < e; ++k) {
      if (a[k] == 0) continue;
      double t = c[id] * a[k];
      for (int i = 0; i < e; ++i) t *= (i == k) ? pw[i][a[i] - 1] : pw[i][a[i]];
      g[k] += t;
    }
  });
}

Poly Poly::restrict_to(int k, double val) const {
  Poly r;
  r.e = e - 1;
  double pv[5] = {1.0, val, val * val, val * val * val, val * val * val * val};
  for_each_exp(e, [&](const int* a, int id) {
    if (c[id] == 0.0) return;
    int nid = 0, m = 0;
    for (int i = 0; i < e; ++i)
      if (i != k) nid += a[i] * pstride(r.e, m++);
    r.c[nid] += c[id] * pv[a[k]];
  });
  return r;
}

Poly Poly::deriv(int k) const {
  Poly r;
  r.e = e;
  for_each_exp(e, [&](const int* a, int id) {
    if (c[id] == 0.0 || a[k] == 0) return;
    r.c[id - pstride(e, k)] += a[k] * c[id];
  });
  return r;
}

void Poly::bounds(const double* lo, const double* hi, double& v, double& spread) const {
  static const double binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0},
                                     {1, 4, 6, 4, 1}};
  double d[125];
  for (int t = 0; t < 125; ++t) d[t] = c[t];
  for (int i = 0; i < e; ++i) {
    const double m = 0.5 * (lo[i] + hi[i]), w = 0.5 * (hi[i] - lo[i]);
    double mp[5] = {1, m, m * m, m * m * m, m * m * m * m};
    double wp[5] = {1, w, w * w, w * w * w, w * w * w * w};
    double nd[125] = {};
    const int st = pstride(e, i);
    for_each_exp(e, [&](const int* a, int id) {
      if (d[id] == 0.0) return;
      for (int b = 0; b <= a[i]; ++b) nd[id - (a[i] - b) * st] += binom[a[i]][b] * mp[a[i] - b] * wp[b] * d[id];
    });
    for (int t = 0; t < 125; ++t) d[t] = nd[t];
  }
  v = d[0];
  spread = 0.0;
  for_each_exp(e, [&](const int*, int id) {
    if (id != 0) spread += std::fabs(d[id]);
  });
}

void Poly::line(int k, const double* xo, double out[5]) const {
  double full[3];
  int m = 0;
  for (int i = 0; i < e; ++i) full[i] = (i == k) ? 1.0 : xo[m++];
  double pw[3][5];
  powers(e, full, pw);
  for (int j = 0; j < 5; ++j) out[j] = 0.0;
  for_each_exp(e, [&](const int* a, int id) {
    if (c[id] == 0.0) return;
    double t = c[id];
    for (int i = 0; i < e; ++i)
      if (i != k) t *= pw[i][a[i]];
    out[a[k]] += t;
  });
}

Poly torus_poly(const double center[3], double R, double r, const double rot[9]) {
  Poly d[3], u[3];
  for (int j = 0; j < 3; ++j) d[j] = poly_coord(j, center[j]);
  for (int i = 0; i < 3; ++i) {
    u[i] = poly_const(3, 0.0);
    for (int j = 0; j < 3; ++j) u[i] = poly_axpy(rot[3 * j + i], d[j], u[i]);
  }
  Poly rho2 = poly_axpy(1.0, poly_mul(u[0], u[0]), poly_mul(u[1], u[1]));
  Poly T = poly_axpy(1.0, rho2, poly_mul(u[2], u[2]));
  T.c[0] += R * R - r * r;
  return poly_axpy(-4.0 * R * R, rho2, poly_mul(T, T));
}

LevelSet LevelSet::restrict_to(int k, double val) const {
  LevelSet r;
  r.poly = poly;
  if (poly)
    r.p = p.restrict_to(k, val);
  else
    r.q = q.restrict_to(k, val);
  return r;
}

void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    // Newton on P_q from the Chebyshev-like initial guess
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // final derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;  // the guesses descend in z, so x ascends
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct GLTable {
  std::vector<double> x, w;
};
static const GLTable& gl(int q) {
  static std::mutex mu;
  static GLTable tabs[33];
  static bool done[33] = {};
  std::lock_guard<std::mutex> lk(mu);
  if (!done[q]) {
    gauss_legendre(q, tabs[q].x, tabs[q].w);
    done[q] = true;
  }
  return tabs[q];
}

// ------------------------------------------------------------------ tests
// +1 / -1 if f provably has that sign on the box, else 0.
static int box_sign(const Quadric& f, const double* lo, const double* hi) {
  double m[3], w[3], g[3];
  for (int i = 0; i < f.e; ++i) {
    m[i] = 0.5 * (lo[i] + hi[i]);
    w[i] = 0.5 * (hi[i] - lo[i]);
  }
  double v = f.eval(m);
  f.grad(m, g);
  double spread = 0.0;
  for (int i = 0; i < f.e; ++i) spread += std::fabs(g[i]) * w[i];
  for (int i = 0; i < f.e; ++i)
    for (int j = 0; j < f.e; ++j) spread += w[i] * std::fabs(f.Q[i][j]) * w[j];
  if (v - spread > 0) return 1;
  if (v + spread < 0) return -1;
  return 0;
}

static int box_sign(const Poly& f, const double* lo, const double* hi) {
  double v, spread;
  f.bounds(lo, hi, v, spread);
  if (v - spread > 0) return 1;
  if (v + spread < 0) return -1;
  return 0;
}

// d f / d x_k is affine; true if it cannot vanish on the box.
static bool monotone(const Quadric& f, int k, const double* lo, const double* hi) {
  double m[3], g[3];
  for (int i = 0; i < f.e; ++i) m[i] = 0.5 * (lo[i] + hi[i]);
  f.grad(m, g);
  double s = 0.0;
  for (int i = 0; i < f.e; ++i) s += std::fabs(2.0 * f.Q[k][i]) * 0.5 * (hi[i] - lo[i]);
  return std::fabs(g[k]) > s;
}

// the Taylor bound of d f / d x_k excludes 0
static bool monotone(const Poly& f, int k, const double* lo, const double* hi) {
  double v, s;
  f.deriv(k).bounds(lo, hi, v, s);
  return std::fabs(v) > s;
}

// |d f/dx_k| >= |grad f| / kSlope on the whole box, from affine bounds.
static bool graph_ok(const Quadric& f, int k, const double* lo, const double* hi) {
  double m[3], w[3], g[3], spread[3];
  for (int i = 0; i < f.e; ++i) {
    m[i] = 0.5 * (lo[i] + hi[i]);
    w[i] = 0.5 * (hi[i] - lo[i]);
  }
  f.grad(m, g);
  for (int i = 0; i < f.e; ++i) {
    double s = 0.0;
    for (int j = 0; j < f.e; ++j) s += std::fabs(2.0 * f.Q[i][j]) * w[j];
    spread[i] = s;
  }
  double low_k = std::fabs(g[k]) - spread[k];
  double up = 0.0;
  for (int i = 0; i < f.e; ++i) up += (std::fabs(g[i]) + spread[i]) * (std::fabs(g[i]) + spread[i]);
  up = std::sqrt(up);
  return low_k > 0 && kSlope * low_k >= up;
}

// the same from the Taylor bounds of the derivatives
static bool graph_ok(const Poly& f, int k, const double* lo, const double* hi) {
  double v[3], s[3];
  for (int i = 0; i < f.e; ++i) f.deriv(i).bounds(lo, hi, v[i], s[i]);
  double low_k = std::fabs(v[k]) - s[k];
  double up = 0.0;
  for (int i = 0; i < f.e; ++i) up += (std::fabs(v[i]) + s[i]) * (std::fabs(v[i]) + s[i]);
  up = std::sqrt(up);
  return low_k > 0 && kSlope * low_k >= up;
}

template <class F>
static int choose_axis(const std::vector<F>& fs, const double* lo, const double* hi, int e) {
  double m[3], score[3] = {0, 0, 0};
  for (int i = 0; i < e; ++i) m[i] = 0.5 * (lo[i] + hi[i]);
  for (const F& f : fs) {
    double g[3];
    f.grad(m, g);
    double nrm = 0.0;
    for (int i = 0; i < e; ++i) nrm += g[i] * g[i];
    nrm = std::sqrt(nrm);
    if (nrm > 0)
      for (int i = 0; i < e; ++i) score[i] += std::fabs(g[i]) / nrm;
  }
  double best = score[0];
  for (int i = 1; i < e; ++i) best = std::max(best, score[i]);
  for (int i = 0; i < e; ++i)
    if (score[i] >= best * (1.0 - kTie)) return i;
  return 0;
}

// Roots of alpha t^2 + beta t + gamma strictly inside (lo, hi); NaN if absent.
static void quad_roots(double alpha, double beta, double gamma, double lo, double hi, double r[2]) {
  r[0] = r[1] = kNaN;
  if (std::fabs(alpha) <= 1e-300) {
    if (beta != 0) r[0] = -gamma / beta;
  } else {
    double disc = beta * beta - 4.0 * alpha * gamma;
    if (disc >= 0) {
      double sq = std::sqrt(disc);
      double qq = -0.5 * (beta + (beta >= 0 ? sq : -sq));
      r[0] = qq / alpha;
      if (qq != 0) r[1] = gamma / qq;
    }
  }
  for (int i = 0; i < 2; ++i)
    if (!(r[i] > lo && r[i] < hi)) r[i] = kNaN;
}

// f along x_k at a base point xo (e-1 coordinates): alpha t^2 + beta t + gamma.
static void line_coeffs(const Quadric& f, int k, const double* xo, double& al, double& be, double& ga) {
  int keep[3], m = 0;
  for (int i = 0; i < f.e; ++i)
    if (i != k) keep[m++] = i;
  al = f.Q[k][k];
  be = f.b[k];
  for (int i = 0; i < m; ++i) be += 2.0 * xo[i] * f.Q[keep[i]][k];
  ga = f.c;
  for (int i = 0; i < m; ++i) {
    ga += f.b[keep[i]] * xo[i];
    for (int j = 0; j < m; ++j) ga += xo[i] * f.Q[keep[i]][keep[j]] * xo[j];
  }
}

// The root in (lo, hi) of the polynomial sum_j a_j t^j (degree <= deg), known
// to be monotone there, by bisection to the last bit; NaN where the two ends
// do not differ in sign.
static double monotone_root(const double* a, int deg, double lo, double hi) {
  double fa = horner(a, deg, lo), fb = horner(a, deg, hi);
  if (fa == 0.0 || fb == 0.0 || (fa < 0) == (fb < 0)) return kNaN;
  double x0 = lo, x1 = hi;
  for (int it = 0; it < 1100; ++it) {
    double m = 0.5 * (x0 + x1);
    if (m <= x0 || m >= x1) break;
    double fm = horner(a, deg, m);
    if ((fm < 0) == (fa < 0)) {
      x0 = m;
      fa = fm;
    } else {
      x1 = m;
    }
  }
  return 0.5 * (x0 + x1);
}

// Sign-changing roots of sum_j a_j t^j inside (lo, hi): the derivative's roots
// cut the interval into monotone pieces; a piece whose ends differ in sign
// holds one root.
static void poly1_roots(const double* a, double lo, double hi, std::vector<double>& out) {
  int deg = 4;
  while (deg > 0 && a[deg] == 0.0) --deg;
  if (deg == 0) return;
  if (deg == 1) {
    double t = -a[0] / a[1];
    if (t > lo && t < hi) out.push_back(t);
    return;
  }
  double da[5] = {0, 0, 0, 0, 0};
  for (int j = 1; j <= deg; ++j) da[j - 1] = j * a[j];
  std::vector<double> cuts = {lo};
  poly1_roots(da, lo, hi, cuts);
  cuts.push_back(hi);
  for (size_t s = 0; s + 1 < cuts.size(); ++s) {
    double f0 = horner(a, deg, cuts[s]), f1 = horner(a, deg, cuts[s + 1]);
    if (f0 != 0.0 && f1 != 0.0 && (f0 < 0) != (f1 < 0)) out.push_back(monotone_root(a, deg, cuts[s], cuts[s + 1]));
  }
}

// Roots along x_k at xo where f is monotone along x_k: kLineRoots slots, NaN = none.
template <class F>
struct RootTraits;
template <>
struct RootTraits<Quadric> {
  static constexpr int kLineRoots = 2;
  static constexpr int kSplitDepth = kMaxDepth;
  static void line(const Quadric& f, int k, const double* xo, double lo, double hi, double* r) {
    double al, be, ga;
    line_coeffs(f, k, xo, al, be, ga);
    quad_roots(al, be, ga, lo, hi, r);
  }
  static void interval(const Quadric& f, double lo, double hi, std::vector<double>& out) {
    double r[2];
    quad_roots(f.Q[0][0], f.b[0], f.c, lo, hi, r);
    out.push_back(r[0]);
    out.push_back(r[1]);
  }
};
template <>
struct RootTraits<Poly> {
  static constexpr int kLineRoots = 1;
  static constexpr int kSplitDepth = kPolySplitDepth;
  static void line(const Poly& f, int k, const double* xo, double lo, double hi, double* r) {
    double a[5];
    f.line(k, xo, a);
    r[0] = monotone_root(a, 4, lo, hi);
  }
  static void interval(const Poly& f, double lo, double hi, std::vector<double>& out) {
    poly1_roots(f.c, lo, hi, out);
  }
};

static void tensor_gauss(const double* lo, const double* hi, int e, int q, NodeSet& out) {
  const GLTable& t = gl(q);
  size_t base = out.w.size();
  size_t P = 1;
  for (int i = 0; i < e; ++i) P *= q;
  out.w.resize(base + P);
  out.x.resize((base + P) * e);
  for (size_t p = 0; p < P; ++p) {
    size_t rem = p;
    double wt = 1.0;
    int idx[3];
    for (int i = e - 1; i >= 0; --i) {
      idx[i] = rem % q;
      rem /= q;
    }
    for (int i = 0; i < e; ++i) {
      double mid = 0.5 * (lo[i] + hi[i]), half = 0.5 * (hi[i] - lo[i]);
      out.x[(base + p) * e + i] = mid + half * t.x[idx[i]];
      wt *= half * t.w[idx[i]];
    }
    out.w[base + p] = wt;
  }
}

// Cut [lo_k, hi_k] at the roots (nr per base point, NaN = none) of every base
// point and put q Gauss points on each piece; all pieces are kept.
static void segments(const NodeSet& base, int k, double lo_k, double hi_k,
                     const std::vector<double>& roots, int nr, int q, int e, NodeSet& out) {
  const GLTable& t = gl(q);
  std::vector<double> br(nr + 2);
  size_t P = base.size();
  for (size_t p = 0; p < P; ++p) {
    br[0] = lo_k;
    for (int j = 0; j < nr; ++j) {
      double r = roots[p * nr + j];
      br[j + 1] = std::isnan(r) ? hi_k : r;
    }
    br[nr + 1] = hi_k;
    std::sort(br.begin(), br.end());
    for (int s = 0; s < nr + 1; ++s) {
      double a = br[s], b = br[s + 1];
      double mid = 0.5 * (a + b), half = 0.5 * (b - a);
      for (int g = 0; g < q; ++g) {
        double wt = base.w[p] * half * t.w[g];
        if (wt == 0.0) continue;
        int m = 0;
        for (int i = 0; i < e; ++i) {
          if (i == k)
            out.x.push_back(mid + half * t.x[g]);
          else
            out.x.push_back(base.x[p * (e - 1) + (m++)]);
        }
        out.w.push_back(wt);
      }
    }
  }
}

template <class F>
static void split_rule(const double* lo, const double* hi, int e, const std::vector<F>& funcs, int q, int depth,
                       NodeSet& out);

template <class F>
static void bisect_split(const double* lo, const double* hi, int e, const std::vector<F>& funcs, int q, int depth,
                         NodeSet& out) {
  double mid[3];
  for (int i = 0; i < e; ++i) mid[i] = 0.5 * (lo[i] + hi[i]);
  for (int code = 0; code < (1 << e); ++code) {
    double a[3], b[3];
    for (int i = 0; i < e; ++i) {
      if ((code >> i) & 1) {
        a[i] = mid[i];
        b[i] = hi[i];
      } else {
        a[i] = lo[i];
        b[i] = mid[i];
      }
    }
    split_rule(a, b, e, funcs, q, depth + 1, out);
  }
}

// Nodes on the box for integrands smooth away from the zero sets of funcs.
template <class F>
static void split_rule(const double* lo, const double* hi, int e, const std::vector<F>& funcs, int q, int depth,
                       NodeSet& out) {
  using RT = RootTraits<F>;
  out.e = e;
  std::vector<F> live;
  for (const F& f : funcs)
    if (box_sign(f, lo, hi) == 0) live.push_back(f);
  if (live.empty()) {
    tensor_gauss(lo, hi, e, q, out);
    return;
  }
  if (e == 1) {
    std::vector<double> roots;
    for (const F& f : live) RT::interval(f, lo[0], hi[0], roots);
    NodeSet base;
    base.e = 0;
    base.w.push_back(1.0);
    segments(base, 0, lo[0], hi[0], roots, (int)roots.size(), q, 1, out);
    return;
  }
  int k = choose_axis(live, lo, hi, e);
  bool ok = true;
  for (const F& f : live) ok = ok && monotone(f, k, lo, hi);
  if (!ok) {
    if (depth < RT::kSplitDepth) {
      bisect_split(lo, hi, e, funcs, q, depth, out);
      return;
    }
    std::vector<F> keep;
    for (const F& f : live)
      if (monotone(f, k, lo, hi)) keep.push_back(f);
    live.swap(keep);
    if (live.empty()) {
      tensor_gauss(lo, hi, e, q, out);
      return;
    }
  }
  double blo[3], bhi[3];
  int m = 0;
  for (int i = 0; i < e; ++i)
    if (i != k) {
      blo[m] = lo[i];
      bhi[m] = hi[i];
      ++m;
    }
  std::vector<F> faces;
  for (const F& f : live) {
    faces.push_back(f.restrict_to(k, lo[k]));
    faces.push_back(f.restrict_to(k, hi[k]));
  }
  NodeSet base;
  split_rule(blo, bhi, e - 1, faces, q, 0, base);
  const int per = RT::kLineRoots;
  int nr = per * (int)live.size();
  std::vector<double> roots(base.size() * nr);
  for (size_t p = 0; p < base.size(); ++p)
    for (size_t j = 0; j < live.size(); ++j) RT::line(live[j], k, &base.x[p * (e - 1)], lo[k], hi[k], &roots[p * nr + per * j]);
  segments(base, k, lo[k], hi[k], roots, nr, q, e, out);
}

// Where the volume rule goes: expanded nodes, or line pieces.
struct NodeSink {
  NodeSet& vol;
  void full_box(const double* lo, const double* hi, int e, int q) { tensor_gauss(lo, hi, e, q, vol); }
  void piece(const double* xo, int k, double a, double b, double wbase, int e, int q) {
    const GLTable& t = gl(q);
    double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    for (int gq = 0; gq < q; ++gq) {
      double wt = wbase * half * t.w[gq];
      if (wt == 0.0) continue;
      int c3 = 0;
      for (int i = 0; i < e; ++i) vol.x.push_back(i == k ? mid + half * t.x[gq] : xo[c3++]);
      vol.w.push_back(wt);
    }
  }
};

struct PieceSink {
  std::vector<LinePiece>& vol;
  void full_box(const double* lo, const double* hi, int e, int q) {
    // the tensor rule as pieces along the last axis over the tensor rule of
    // the first two
    const GLTable& t = gl(q);
    const double m0 = 0.5 * (lo[0] + hi[0]), h0 = 0.5 * (hi[0] - lo[0]);
    const double m1 = 0.5 * (lo[1] + hi[1]), h1 = 0.5 * (hi[1] - lo[1]);
    (void)e;
    for (int i0 = 0; i0 < q; ++i0)
      for (int i1 = 0; i1 < q; ++i1) {
        LinePiece lp;
        lp.xo[0] = m0 + h0 * t.x[i0];
        lp.xo[1] = m1 + h1 * t.x[i1];
        lp.a = lo[2];
        lp.b = hi[2];
        lp.w = (h0 * t.w[i0]) * (h1 * t.w[i1]);
        lp.k = 2;
        lp.pad_ = 0;
        vol.push_back(lp);
      }
  }
  void piece(const double* xo, int k, double a, double b, double wbase, int, int) {
    if (wbase == 0.0 || b == a) return;
    LinePiece lp;
    lp.xo[0] = xo[0];
    lp.xo[1] = xo[1];
    lp.a = a;
    lp.b = b;
    lp.w = wbase;
    lp.k = k;
    lp.pad_ = 0;
    vol.push_back(lp);
  }
};

template <class F, class Sink>
static void region_impl(const double* lo, const double* hi, int e, const F& psi, int q, Sink& vol,
                        SurfaceSet* surf, int depth) {
  using RT = RootTraits<F>;
  int s = box_sign(psi, lo, hi);
  if (s > 0) {
    vol.full_box(lo, hi, e, q);
    return;
  }
  if (s < 0) return;
  double m[3], g[3];
  for (int i = 0; i < e; ++i) m[i] = 0.5 * (lo[i] + hi[i]);
  psi.grad(m, g);
  double best = 0.0;
  for (int i = 0; i < e; ++i) best = std::max(best, std::fabs(g[i]));
  int k = 0;
  for (int i = 0; i < e; ++i)
    if (std::fabs(g[i]) >= best * (1.0 - kTie)) {
      k = i;
      break;
    }
  if (!graph_ok(psi, k, lo, hi)) {
    if (depth < kMaxDepth) {
      for (int code = 0; code < (1 << e); ++code) {
        double a[3], b[3];
        for (int i = 0; i < e; ++i) {
          if ((code >> i) & 1) {
            a[i] = m[i];
            b[i] = hi[i];
          } else {
            a[i] = lo[i];
            b[i] = m[i];
          }
        }
        region_impl(a, b, e, psi, q, vol, surf, depth + 1);
      }
      return;
    }
    if (psi.eval(m) > 0) vol.full_box(lo, hi, e, q);
    return;
  }
  double blo[3], bhi[3];
  int mm = 0;
  for (int i = 0; i < e; ++i)
    if (i != k) {
      blo[mm] = lo[i];
      bhi[mm] = hi[i];
      ++mm;
    }
  std::vector<F> faces = {psi.restrict_to(k, lo[k]), psi.restrict_to(k, hi[k])};
  NodeSet base;
  split_rule(blo, bhi, e - 1, faces, q, 0, base);
  for (size_t p = 0; p < base.size(); ++p) {
    const double* xo = &base.x[p * (e - 1)];
    double r[2];
    RT::line(psi, k, xo, lo[k], hi[k], r);
    // psi is monotone along x_k here: at most one root on the interval
    double root = (RT::kLineRoots == 1 || !std::isnan(r[0])) ? r[0] : r[1];
    double br[3] = {lo[k], std::isnan(root) ? hi[k] : root, hi[k]};
    std::sort(br, br + 3);
    for (int sgi = 0; sgi < 2; ++sgi) {
      double a = br[sgi], b = br[sgi + 1];
      double mid = 0.5 * (a + b);
      double xm[3];
      int c2 = 0;
      for (int i = 0; i < e; ++i) xm[i] = (i == k) ? mid : xo[c2++];
      if (!(psi.eval(xm) > 0)) continue;
      vol.piece(xo, k, a, b, base.w[p], e, q);
    }
    if (surf && e == 3 && !std::isnan(root)) {
      double xs[3], gs[3];
      int c4 = 0;
      for (int i = 0; i < 3; ++i) xs[i] = (i == k) ? root : xo[c4++];
      psi.grad(xs, gs);
      double gn = std::sqrt(gs[0] * gs[0] + gs[1] * gs[1] + gs[2] * gs[2]);
      for (int i = 0; i < 3; ++i) {
        surf->x.push_back(xs[i]);
        surf->n.push_back(-gs[i] / gn);
      }
      surf->w.push_back(base.w[p] * gn / std::fabs(gs[k]));
    }
  }
}

void region_rules(const double* lo, const double* hi, int e, const LevelSet& psi, int q, NodeSet& vol,
                  SurfaceSet* surf, int depth) {
  vol.e = e;
  NodeSink sink{vol};
  if (psi.poly)
    region_impl(lo, hi, e, psi.p, q, sink, surf, depth);
  else
    region_impl(lo, hi, e, psi.q, q, sink, surf, depth);
}

void region_pieces(const double* lo, const double* hi, const LevelSet& psi, int q, std::vector<LinePiece>& vol,
                   SurfaceSet* surf) {
  PieceSink sink{vol};
  if (psi.poly)
    region_impl(lo, hi, 3, psi.p, q, sink, surf, 0);
  else
    region_impl(lo, hi, 3, psi.q, q, sink, surf, 0);
}

}  // namespace cc
