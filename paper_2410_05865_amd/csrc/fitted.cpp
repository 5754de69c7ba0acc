// The paper's boundary fitting (Sec. 3.1) on cut cells, as a check of the
// exact geometry the solver uses (the geometry accuracy test of Sec. 6.1,
// Table 1).  Per cut cell: points of the exact boundary inside the cell (the
// surface nodes of a kFitQ-point height-function rule), the height axis of
// the patch's mean normal, a least-squares quadratic height function in
// cell-centred coordinates scaled by h (minimum-norm, singular values below
// kFitRcond times the largest dropped), and the fitted region as a quadric
// integrated with the same height-function rule as the exact one.
#include <algorithm>
#include <cmath>
#include <vector>

#include "level.hpp"
#include "quadrature.hpp"

namespace cc {

namespace {

constexpr int kFitQ = 4;
constexpr double kFitRcond = 1e-12;

// Minimum-norm least squares of A x = b (A: m x 6, row-major) by one-sided
// Jacobi SVD: columns of A rotated until orthogonal, V accumulating the
// rotations; x = sum over kept singular values of (u_i . b / s_i) v_i.
void lstsq6(std::vector<double> A, const std::vector<double>& b, double x[6]) {
  const int m = (int)b.size(), n = 6;
  double V[6][6] = {};
  for (int i = 0; i < n; ++i) V[i][i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, bb = 0.0, g = 0.0;
        for (int r = 0; r < m; ++r) {
          a += A[r * n + p] * A[r * n + p];
          bb += A[r * n + q] * A[r * n + q];
          g += A[r * n + p] * A[r * n + q];
        }
        if (g == 0.0) continue;
        off = std::max(off, std::fabs(g) / std::sqrt(a * bb));
        double zeta = (bb - a) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < m; ++r) {
          double ap = A[r * n + p], aq = A[r * n + q];
          A[r * n + p] = c * ap - s * aq;
          A[r * n + q] = s * ap + c * aq;
        }
        for (int r = 0; r < n; ++r) {
          double vp = V[r][p], vq = V[r][q];
          V[r][p] = c * vp - s * vq;
          V[r][q] = s * vp + c * vq;
        }
      }
    if (off < 1e-15) break;
  }
  double sv[6], smax = 0.0;
  for (int i = 0; i < n; ++i) {
    double t = 0.0;
    for (int r = 0; r < m; ++r) t += A[r * n + i] * A[r * n + i];
    sv[i] = std::sqrt(t);
    smax = std::max(smax, sv[i]);
  }
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!(sv[i] > kFitRcond * smax)) continue;
    double ub = 0.0;
    for (int r = 0; r < m; ++r) ub += A[r * n + i] * b[r];   // (s_i u_i) . b
    const double coef = ub / (sv[i] * sv[i]);
    for (int j = 0; j < n; ++j) x[j] += coef * V[j][i];
  }
}

void averages(const double* lo, const double* hi, const LevelSet& psi, const FieldDesc& u, double out[4]) {
  NodeSet vn;
  SurfaceSet sn;
  region_rules(lo, hi, 3, psi, kQuadOrder, vn, &sn);
  double V = 0.0, A = 0.0, iv = 0.0, is = 0.0;
  for (size_t q = 0; q < vn.size(); ++q) {
    V += vn.w[q];
    iv += vn.w[q] * field_value(u, vn.x[3 * q], vn.x[3 * q + 1], vn.x[3 * q + 2], 0);
  }
  for (size_t q = 0; q < sn.w.size(); ++q) {
    A += sn.w[q];
    is += sn.w[q] * field_value(u, sn.x[3 * q], sn.x[3 * q + 1], sn.x[3 * q + 2], 0);
  }
  out[0] = V;
  out[1] = A;
  out[2] = V > 0 ? iv / V : std::nan("");
  out[3] = A > 0 ? is / A : std::nan("");
}

}  // namespace

// axis = -1 (and NaN results) where the exact patch gives fewer than 6 points.
void fit_cut_cells(const LevelHost& L, const DomainSpec& dom, const FieldDesc& u, int* cell, int* axis, double* coef,
                   double* exact, double* fitted) {
  std::vector<int> cuts;
  for (const auto& kv : L.cut) cuts.push_back(kv.first);
  std::sort(cuts.begin(), cuts.end());
#pragma omp parallel for schedule(dynamic, 8)
  for (long t = 0; t < (long)cuts.size(); ++t) {
    const int p = cuts[t];
    const LevelSet& psi = dom.obst[L.cut.at(p).obst].ls;
    int ii[3];
    L.ijk(p, ii[0], ii[1], ii[2]);
    double lo[3], hi[3], c[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = L.origin[a] + L.h * ii[a];
      hi[a] = lo[a] + L.h;
      c[a] = 0.5 * (lo[a] + hi[a]);
    }
    if (cell) cell[t] = p;
    double ex[4];
    averages(lo, hi, psi, u, ex);
    if (exact)
      for (int k = 0; k < 4; ++k) exact[4 * t + k] = ex[k];
    NodeSet vn;
    SurfaceSet sn;
    region_rules(lo, hi, 3, psi, kFitQ, vn, &sn);
    const int np = (int)sn.w.size();
    if (np < 6) {
      if (axis) axis[t] = -1;
      for (int k = 0; k < 6 && coef; ++k) coef[6 * t + k] = std::nan("");
      for (int k = 0; k < 4 && fitted; ++k) fitted[4 * t + k] = std::nan("");
      continue;
    }
    double nbar[3] = {0, 0, 0};
    for (int q = 0; q < np; ++q)
      for (int a = 0; a < 3; ++a) nbar[a] += sn.w[q] * sn.n[3 * q + a];
    const double amax = std::max(std::fabs(nbar[0]), std::max(std::fabs(nbar[1]), std::fabs(nbar[2])));
    int w = 0;
    while (std::fabs(nbar[w]) < amax * (1.0 - kTie)) ++w;   // near-ties go to the lowest axis
    const int u0 = w == 0 ? 1 : 0, v0 = w == 2 ? 1 : 2;
    const double h = L.h;
    std::vector<double> A((size_t)np * 6), b(np);
    for (int q = 0; q < np; ++q) {
      const double U = (sn.x[3 * q + u0] - c[u0]) / h, Vv = (sn.x[3 * q + v0] - c[v0]) / h;
      double* r = &A[(size_t)q * 6];
      r[0] = U * U;
      r[1] = U * Vv;
      r[2] = Vv * Vv;
      r[3] = U;
      r[4] = Vv;
      r[5] = 1.0;
      b[q] = (sn.x[3 * q + w] - c[w]) / h;
    }
    double k6[6];
    lstsq6(A, b, k6);
    // s (W - p(U, V)) h as a quadric in x; Omega lies toward -nbar
    const double s = -nbar[w] > 0 ? 1.0 : -1.0;
    LevelSet fit;
    Quadric& Q = fit.q;
    Q.e = 3;
    const double cu = c[u0], cv = c[v0], cw = c[w];
    Q.Q[u0][u0] = -s * k6[0] / h;
    Q.Q[v0][v0] = -s * k6[2] / h;
    Q.Q[u0][v0] = Q.Q[v0][u0] = -s * k6[1] / (2.0 * h);
    Q.b[u0] = -s * (-2.0 * k6[0] * cu / h - k6[1] * cv / h + k6[3]);
    Q.b[v0] = -s * (-2.0 * k6[2] * cv / h - k6[1] * cu / h + k6[4]);
    Q.b[w] = s;
    Q.c = -s * (k6[0] * cu * cu / h + k6[1] * cu * cv / h + k6[2] * cv * cv / h - k6[3] * cu - k6[4] * cv + k6[5] * h) -
          s * cw;
    if (axis) axis[t] = w;
    for (int k = 0; k < 6 && coef; ++k) coef[6 * t + k] = k6[k];
    double fi[4];
    averages(lo, hi, fit, u, fi);
    if (fitted)
      for (int k = 0; k < 4; ++k) fitted[4 * t + k] = fi[k];
  }
}

}  // namespace cc
