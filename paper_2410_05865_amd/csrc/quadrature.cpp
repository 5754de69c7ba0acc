// Height-function quadrature on boxes cut by quadrics (see quadrature.hpp).
#include "quadrature.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <mutex>

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

// d f / d x_k is affine; true if it cannot vanish on the box.
static bool monotone(const Quadric& f, int k, const double* lo, const double* hi) {
  double m[3], g[3];
  for (int i = 0; i < f.e; ++i) m[i] = 0.5 * (lo[i] + hi[i]);
  f.grad(m, g);
  double s = 0.0;
  for (int i = 0; i < f.e; ++i) s += std::fabs(2.0 * f.Q[k][i]) * 0.5 * (hi[i] - lo[i]);
  return std::fabs(g[k]) > s;
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

static int choose_axis(const std::vector<Quadric>& fs, const double* lo, const double* hi, int e) {
  double m[3], score[3] = {0, 0, 0};
  for (int i = 0; i < e; ++i) m[i] = 0.5 * (lo[i] + hi[i]);
  for (const Quadric& f : fs) {
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

static void split_rule(const double* lo, const double* hi, int e, const std::vector<Quadric>& funcs,
                       int q, int depth, NodeSet& out);

static void bisect_split(const double* lo, const double* hi, int e, const std::vector<Quadric>& funcs,
                         int q, int depth, NodeSet& out) {
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
static void split_rule(const double* lo, const double* hi, int e, const std::vector<Quadric>& funcs,
                       int q, int depth, NodeSet& out) {
  out.e = e;
  std::vector<Quadric> live;
  for (const Quadric& f : funcs)
    if (box_sign(f, lo, hi) == 0) live.push_back(f);
  if (live.empty()) {
    tensor_gauss(lo, hi, e, q, out);
    return;
  }
  if (e == 1) {
    std::vector<double> roots;
    for (const Quadric& f : live) {
      double r[2];
      quad_roots(f.Q[0][0], f.b[0], f.c, lo[0], hi[0], r);
      roots.push_back(r[0]);
      roots.push_back(r[1]);
    }
    NodeSet base;
    base.e = 0;
    base.w.push_back(1.0);
    segments(base, 0, lo[0], hi[0], roots, (int)roots.size(), q, 1, out);
    return;
  }
  int k = choose_axis(live, lo, hi, e);
  bool ok = true;
  for (const Quadric& f : live) ok = ok && monotone(f, k, lo, hi);
  if (!ok) {
    if (depth < kMaxDepth) {
      bisect_split(lo, hi, e, funcs, q, depth, out);
      return;
    }
    std::vector<Quadric> keep;
    for (const Quadric& f : live)
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
  std::vector<Quadric> faces;
  for (const Quadric& f : live) {
    faces.push_back(f.restrict_to(k, lo[k]));
    faces.push_back(f.restrict_to(k, hi[k]));
  }
  NodeSet base;
  split_rule(blo, bhi, e - 1, faces, q, 0, base);
  int nr = 2 * (int)live.size();
  std::vector<double> roots(base.size() * nr);
  for (size_t p = 0; p < base.size(); ++p)
    for (size_t j = 0; j < live.size(); ++j) {
      double al, be, ga, r[2];
      line_coeffs(live[j], k, &base.x[p * (e - 1)], al, be, ga);
      quad_roots(al, be, ga, lo[k], hi[k], r);
      roots[p * nr + 2 * j] = r[0];
      roots[p * nr + 2 * j + 1] = r[1];
    }
  segments(base, k, lo[k], hi[k], roots, nr, q, e, out);
}

void region_rules(const double* lo, const double* hi, int e, const Quadric& psi, int q, NodeSet& vol,
                  SurfaceSet* surf, int depth) {
  vol.e = e;
  int s = box_sign(psi, lo, hi);
  if (s > 0) {
    tensor_gauss(lo, hi, e, q, vol);
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
        region_rules(a, b, e, psi, q, vol, surf, depth + 1);
      }
      return;
    }
    if (psi.eval(m) > 0) tensor_gauss(lo, hi, e, q, vol);
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
  std::vector<Quadric> faces = {psi.restrict_to(k, lo[k]), psi.restrict_to(k, hi[k])};
  NodeSet base;
  split_rule(blo, bhi, e - 1, faces, q, 0, base);
  const GLTable& t = gl(q);
  for (size_t p = 0; p < base.size(); ++p) {
    const double* xo = &base.x[p * (e - 1)];
    double al, be, ga, r[2];
    line_coeffs(psi, k, xo, al, be, ga);
    quad_roots(al, be, ga, lo[k], hi[k], r);
    double root = std::isnan(r[0]) ? r[1] : r[0];
    double br[3] = {lo[k], std::isnan(root) ? hi[k] : root, hi[k]};
    std::sort(br, br + 3);
    for (int sgi = 0; sgi < 2; ++sgi) {
      double a = br[sgi], b = br[sgi + 1];
      double mid = 0.5 * (a + b), half = 0.5 * (b - a);
      double xm[3];
      int c2 = 0;
      for (int i = 0; i < e; ++i) xm[i] = (i == k) ? mid : xo[c2++];
      if (!(psi.eval(xm) > 0)) continue;
      for (int gq = 0; gq < q; ++gq) {
        double wt = base.w[p] * half * t.w[gq];
        if (wt == 0.0) continue;
        int c3 = 0;
        for (int i = 0; i < e; ++i) vol.x.push_back(i == k ? mid + half * t.x[gq] : xo[c3++]);
        vol.w.push_back(wt);
      }
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

}  // namespace cc
