// Host construction of one grid level; see level.hpp.
#include "level.hpp"

#include <omp.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <deque>
#include <set>
#include <string>

namespace cc {

// ------------------------------------------------------------- monomials
MonoTable::MonoTable() {
  for (auto& a : idx4)
    for (auto& b : a)
      for (auto& c : b) c = -1;
  for (auto& a : idx3)
    for (auto& b : a)
      for (auto& c : b) c = -1;
  int t4 = 0, t3 = 0;
  for (int d = 0; d <= 4; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        int c = d - a - b;
        e4[t4][0] = a;
        e4[t4][1] = b;
        e4[t4][2] = c;
        idx4[a][b][c] = t4++;
        if (d <= 3) {
          e3[t3][0] = a;
          e3[t3][1] = b;
          e3[t3][2] = c;
          idx3[a][b][c] = t3++;
        }
      }
}
const MonoTable& mono() {
  static MonoTable t;
  return t;
}

static const double kBinom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                                    {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};

static double ipowi(int x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

void shift_moments4(const double m[N4], const int d[3], double out[N4]) {
  const MonoTable& T = mono();
  for (int j = 0; j < N4; ++j) {
    const int* a = T.e4[j];
    double s = 0.0;
    for (int b0 = 0; b0 <= a[0]; ++b0)
      for (int b1 = 0; b1 <= a[1]; ++b1)
        for (int b2 = 0; b2 <= a[2]; ++b2)
          s += kBinom[a[0]][b0] * kBinom[a[1]][b1] * kBinom[a[2]][b2] * ipowi(d[0], a[0] - b0) *
               ipowi(d[1], a[1] - b1) * ipowi(d[2], a[2] - b2) * m[T.idx4[b0][b1][b2]];
    out[j] = s;
  }
}

void shift_moments3(const double m[N3], const int d[3], double out[N3]) {
  const MonoTable& T = mono();
  for (int j = 0; j < N3; ++j) {
    const int* a = T.e3[j];
    double s = 0.0;
    for (int b0 = 0; b0 <= a[0]; ++b0)
      for (int b1 = 0; b1 <= a[1]; ++b1)
        for (int b2 = 0; b2 <= a[2]; ++b2)
          s += kBinom[a[0]][b0] * kBinom[a[1]][b1] * kBinom[a[2]][b2] * ipowi(d[0], a[0] - b0) *
               ipowi(d[1], a[1] - b1) * ipowi(d[2], a[2] - b2) * m[T.idx3[b0][b1][b2]];
    out[j] = s;
  }
}

// <xi^a> over the unit cube [-1/2, 1/2]^3
static const std::array<double, N4>& full_moments() {
  static std::array<double, N4> m = [] {
    std::array<double, N4> r{};
    auto mu = [](int k) { return (k % 2) ? 0.0 : 1.0 / ((k + 1) * std::pow(2.0, k)); };
    const MonoTable& T = mono();
    for (int j = 0; j < N4; ++j) r[j] = mu(T.e4[j][0]) * mu(T.e4[j][1]) * mu(T.e4[j][2]);
    return r;
  }();
  return m;
}

const std::vector<int>& LevelHost::members(int p, std::vector<int>& tmp) const {
  auto it = groups.find(p);
  if (it != groups.end()) return it->second;
  tmp.assign(1, p);
  return tmp;
}

// ------------------------------------------------------------- build
void LevelHost::build(const DomainSpec& d, int n_level, double theta, PlgLsqSolver* lsq) {
  dom = &d;
  n = n_level;
  h = 1.0 / n;
  for (int i = 0; i < 3; ++i) origin[i] = d.origin[i];
  for (int i = 0; i < 6; ++i) {
    wall_bc[i] = d.wall_bc[i];
    wall[i] = wall_rows(d.wall_bc[i], d.wall_robin[i][0], d.wall_robin[i][1], h);
  }
  size_t n3 = (size_t)n * n * n;
  // away from the obstacles' claimed cells: interior in the box minus the
  // obstacles, exterior for the interior of one obstacle
  cls.assign(n3, d.inside ? kExterior : kInterior);
  vol.assign(n3, d.inside ? 0.0 : h * h * h);
  owner.assign(n3, -1);
  claim();
  classify();
  merge(theta);
  split();
  rows(lsq);
}

void LevelHost::claim() {
  for (size_t t = 0; t < dom->obst.size(); ++t) {
    const Obstacle& o = dom->obst[t];
    int lo_i[3], hi_i[3];
    for (int a = 0; a < 3; ++a) {
      lo_i[a] = std::max(0, (int)std::floor((o.c[a] - o.R - origin[a]) / h) - 1);
      hi_i[a] = std::min(n - 1, (int)std::floor((o.c[a] + o.R - origin[a]) / h) + 1);
    }
    for (int k = lo_i[2]; k <= hi_i[2]; ++k)
      for (int j = lo_i[1]; j <= hi_i[1]; ++j)
        for (int i = lo_i[0]; i <= hi_i[0]; ++i) {
          int ii[3] = {i, j, k};
          double s = 0.0;
          for (int a = 0; a < 3; ++a) {
            double lo = origin[a] + h * ii[a], hi = lo + h;
            double dd = std::max(std::max(lo - o.c[a], 0.0), o.c[a] - hi);
            s += dd * dd;
          }
          if (!(s < o.R * o.R)) continue;
          int p = idx(i, j, k);
          if (owner[p] >= 0) fail(CC_EGEOM, "a cell meets two obstacles at n=" + std::to_string(n));
          if (i == 0 || i == n - 1 || j == 0 || j == n - 1 || k == 0 || k == n - 1)
            fail(CC_EGEOM, "an obstacle reaches the wall layer at n=" + std::to_string(n));
          owner[p] = (int)t;
        }
  }
}

void LevelHost::classify() {
  std::vector<int> claimed;
  for (size_t p = 0; p < owner.size(); ++p)
    if (owner[p] >= 0) claimed.push_back((int)p);
  const double h3 = h * h * h;
  const MonoTable& T = mono();
  std::vector<CutData> data(claimed.size());
  std::vector<int8_t> ccls(claimed.size());
  std::vector<double> cvol(claimed.size());
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < (long)claimed.size(); ++t) {
    int p = claimed[t];
    int i, j, k;
    ijk(p, i, j, k);
    double lo[3] = {origin[0] + h * i, origin[1] + h * j, origin[2] + h * k};
    double hi[3] = {lo[0] + h, lo[1] + h, lo[2] + h};
    const Obstacle& o = dom->obst[owner[p]];
    NodeSet vn;
    SurfaceSet sn;
    region_rules(lo, hi, 3, o.ls, kQuadOrder, vn, &sn);
    double V = 0.0;
    for (double w : vn.w) V += w;
    if (V < 1e-12 * h3) {
      ccls[t] = kExterior;
      cvol[t] = 0.0;
      continue;
    }
    if (V > (1.0 - 1e-12) * h3) {
      ccls[t] = kInterior;
      cvol[t] = h3;
      continue;
    }
    ccls[t] = kCut;
    cvol[t] = V;
    CutData& cd = data[t];
    cd.obst = owner[p];
    cd.vol = V;
    double xc[3] = {lo[0] + 0.5 * h, lo[1] + 0.5 * h, lo[2] + 0.5 * h};
    for (int a = 0; a < N4; ++a) cd.m[a] = cd.sm[a] = 0.0;
    for (int dd = 0; dd < 3; ++dd)
      for (int a = 0; a < N3; ++a) cd.sn[dd][a] = 0.0;
    for (size_t q = 0; q < vn.size(); ++q) {
      double xi[3];
      for (int a = 0; a < 3; ++a) xi[a] = (vn.x[3 * q + a] - xc[a]) / h;
      for (int a = 0; a < N4; ++a)
        cd.m[a] += vn.w[q] * ipow(xi[0], T.e4[a][0]) * ipow(xi[1], T.e4[a][1]) * ipow(xi[2], T.e4[a][2]);
    }
    for (int a = 0; a < N4; ++a) cd.m[a] /= V;
    double A = 0.0;
    for (double w : sn.w) A += w;
    cd.area = A;
    for (size_t q = 0; q < sn.w.size(); ++q) {
      double xi[3];
      for (int a = 0; a < 3; ++a) xi[a] = (sn.x[3 * q + a] - xc[a]) / h;
      for (int a = 0; a < N4; ++a) {
        double mv = ipow(xi[0], T.e4[a][0]) * ipow(xi[1], T.e4[a][1]) * ipow(xi[2], T.e4[a][2]);
        cd.sm[a] += sn.w[q] * mv;
        if (a < N3)
          for (int dd = 0; dd < 3; ++dd) cd.sn[dd][a] += sn.w[q] * sn.n[3 * q + dd] * mv;
      }
    }
    if (A > 0) {
      for (int a = 0; a < N4; ++a) cd.sm[a] /= A;
      for (int dd = 0; dd < 3; ++dd)
        for (int a = 0; a < N3; ++a) cd.sn[dd][a] /= A;
    }
  }
  for (size_t t = 0; t < claimed.size(); ++t) {
    int p = claimed[t];
    cls[p] = ccls[t];
    vol[p] = cvol[t];
    if (ccls[t] == kCut) cut[p] = data[t];
  }
}

double LevelHost::face_area(int p, int d, int side) const {
  int ii[3];
  ijk(p, ii[0], ii[1], ii[2]);
  int qq[3] = {ii[0], ii[1], ii[2]};
  qq[d] += side;
  if (qq[d] < 0 || qq[d] >= n) return 0.0;
  int q = idx(qq[0], qq[1], qq[2]);
  if (cls[p] == kExterior || cls[q] == kExterior) return 0.0;
  int t = owner[p] >= 0 ? owner[p] : owner[q];
  if (t < 0) return h * h;
  double xf = origin[d] + h * (ii[d] + (side > 0 ? 1 : 0));
  LevelSet f2 = dom->obst[t].ls.restrict_to(d, xf);
  double lo[2], hi[2];
  int m = 0;
  for (int a = 0; a < 3; ++a)
    if (a != d) {
      lo[m] = origin[a] + h * ii[a];
      hi[m] = lo[m] + h;
      ++m;
    }
  NodeSet vn;
  region_rules(lo, hi, 2, f2, kQuadOrder, vn, nullptr);
  double s = 0.0;
  for (double w : vn.w) s += w;
  return s;
}

static const int kNeigh[6][2] = {{0, -1}, {0, 1}, {1, -1}, {1, 1}, {2, -1}, {2, 1}};

void LevelHost::merge(double theta) {
  const double h3 = h * h * h;
  size_t n3 = cls.size();
  host.resize(n3);
  for (size_t p = 0; p < n3; ++p) host[p] = (cls[p] == kExterior) ? -1 : (int)p;
  auto neighbour = [&](int p, int d, int s) {
    int ii[3];
    ijk(p, ii[0], ii[1], ii[2]);
    ii[d] += s;
    if (ii[d] < 0 || ii[d] >= n) return -1;
    return idx(ii[0], ii[1], ii[2]);
  };
  std::vector<int> small;
  for (const auto& kv : cut)
    if (vol[kv.first] < theta * h3) small.push_back(kv.first);
  std::vector<int> pending;
  for (int p : small) {
    std::vector<std::pair<double, int>> cands;
    for (const auto& ds : kNeigh) {
      int q = neighbour(p, ds[0], ds[1]);
      if (q < 0 || cls[q] == kExterior || vol[q] < theta * h3) continue;
      double a = face_area(p, ds[0], ds[1]);
      if (a > 0) cands.push_back({a, q});
    }
    if (!cands.empty()) {
      double amax = 0.0;
      for (auto& c : cands) amax = std::max(amax, c.first);
      int best = -1;
      for (auto& c : cands)
        if (c.first >= amax * (1.0 - 1e-10) && (best < 0 || c.second < best)) best = c.second;
      host[p] = best;
    } else {
      pending.push_back(p);
    }
  }
  for (int p : pending) {
    std::set<int> group;
    group.insert(p);
    for (size_t q = 0; q < n3; ++q)
      if (host[q] == p) group.insert((int)q);
    double gv = 0.0;
    for (int q : group) gv += vol[q];
    std::set<int> seen = {p};
    std::deque<int> queue = {p};
    while (!queue.empty() && gv < theta * h3) {
      int u = queue.front();
      queue.pop_front();
      for (const auto& ds : kNeigh) {
        int v = neighbour(u, ds[0], ds[1]);
        if (v < 0 || seen.count(v) || cls[v] == kExterior) continue;
        if (face_area(u, ds[0], ds[1]) <= 0) continue;
        seen.insert(v);
        queue.push_back(v);
        int w = host[v];
        std::set<int> mem = {w, v};
        for (size_t q = 0; q < n3; ++q)
          if (host[q] == w) mem.insert((int)q);
        for (int q : mem) {
          if (!group.count(q)) {
            group.insert(q);
            gv += vol[q];
          }
          host[q] = p;
        }
        if (gv >= theta * h3) break;
      }
    }
    if (gv < theta * h3) fail(CC_EGEOM, "merging could not reach a theta-proper cell");
    for (int q : group) host[q] = p;
  }
  groups.clear();
  n_merged = 0;
  for (size_t q = 0; q < n3; ++q)
    if (host[q] >= 0 && host[q] != (int)q) {
      groups[host[q]].push_back((int)q);
      ++n_merged;
    }
  for (auto& kv : groups) {
    kv.second.push_back(kv.first);
    std::sort(kv.second.begin(), kv.second.end());
  }
}

bool LevelHost::regular_ok(int p) const {
  if (!plain[p]) return false;
  int ii[3];
  ijk(p, ii[0], ii[1], ii[2]);
  for (int d = 0; d < 3; ++d)
    for (int o : {-2, -1, 1, 2}) {
      int c = ii[d] + o;
      int q[3] = {ii[0], ii[1], ii[2]};
      if (c >= 0 && c < n) {
        q[d] = c;
        if (!plain[idx(q[0], q[1], q[2])]) return false;
      } else {
        int t0 = (c >= n) ? n - 4 : 0;
        for (int t = t0; t < t0 + 4; ++t) {
          q[d] = t;
          if (!plain[idx(q[0], q[1], q[2])]) return false;
        }
      }
    }
  return true;
}

void LevelHost::split() {
  size_t n3 = cls.size();
  plain.assign(n3, 0);
  unknowns.clear();
  for (size_t p = 0; p < n3; ++p)
    if (host[p] == (int)p) {
      unknowns.push_back((int)p);
      if (cls[p] == kInterior && !groups.count((int)p)) plain[p] = 1;
    }
  type.assign(n3, kNone);
#pragma omp parallel for schedule(static)
  for (long t = 0; t < (long)unknowns.size(); ++t) {
    int p = unknowns[t];
    type[p] = regular_ok(p) ? kPhi1 : kPhi2;
  }
  phi2.clear();
  for (int p : unknowns)
    if (type[p] == kPhi2) phi2.push_back(p);
}

// ------------------------------------------------------------- PLG search
namespace {
struct Numbering {
  int k;
  int key[5];
  int pts[5];
};

std::vector<std::array<int, 3>> shift_order() {
  std::vector<std::array<int, 3>> v;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) v.push_back({a, b, c});
  std::sort(v.begin(), v.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
    int sx = x[0] + x[1] + x[2], sy = y[0] + y[1] + y[2];
    if (sx != sy) return sx < sy;
    if (x[0] != y[0]) return x[0] > y[0];
    if (x[1] != y[1]) return x[1] > y[1];
    return x[2] > y[2];
  });
  return v;
}

// Contiguous-growth numberings of lo..lo+4, sorted by (position of i, then the
// signed offsets -sgn (p_j - i) in increasing order).
void axis_numberings(int i, int lo, int sgn, std::vector<Numbering>& out) {
  out.clear();
  for (int start = lo; start < lo + 5; ++start) {
    int below = start - lo, above = 4 - below;
    for (int code = 0; code < 16; ++code) {
      int ups = 0;
      for (int b = 0; b < 4; ++b) ups += (code >> (3 - b)) & 1 ? 0 : 1;  // bit 0 -> 'F' (up)
      if (ups != above) continue;
      Numbering nb;
      int a = start, bb = start;
      nb.pts[0] = start;
      for (int b = 0; b < 4; ++b) {
        bool up = !((code >> (3 - b)) & 1);
        if (up)
          nb.pts[b + 1] = ++bb;
        else
          nb.pts[b + 1] = --a;
      }
      nb.k = -1;
      for (int t = 0; t < 5; ++t) {
        if (nb.pts[t] == i) nb.k = t;
        nb.key[t] = -sgn * (nb.pts[t] - i);
      }
      out.push_back(nb);
    }
  }
  std::sort(out.begin(), out.end(), [](const Numbering& x, const Numbering& y) {
    if (x.k != y.k) return x.k < y.k;
    for (int t = 0; t < 5; ++t)
      if (x.key[t] != y.key[t]) return x.key[t] < y.key[t];
    return false;
  });
}
}  // namespace

void LevelHost::plg_select(int p, int cells[kPLG]) const {
  static const std::vector<std::array<int, 3>> shifts = shift_order();
  const MonoTable& T = mono();
  int ii[3];
  ijk(p, ii[0], ii[1], ii[2]);
  double xc[3] = {origin[0] + h * (ii[0] + 0.5), origin[1] + h * (ii[1] + 0.5), origin[2] + h * (ii[2] + 0.5)};
  int sgn[3] = {1, 1, 1};
  int bt = -1;
  double best = 0.0;
  for (size_t t = 0; t < dom->obst.size(); ++t) {
    const Obstacle& o = dom->obst[t];
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (xc[a] - o.c[a]) * (xc[a] - o.c[a]);
    double dist = std::sqrt(d2) - o.R;
    if (bt < 0 || dist < best) {
      best = dist;
      bt = (int)t;
    }
  }
  if (bt >= 0) {
    const Obstacle& o = dom->obst[bt];
    // the direction into Omega: the level set's gradient (for a quadric
    // (x - c)^T A (x - c) - 1, its half, A (x - c))
    double g[3], gn = 0.0;
    if (o.ls.poly) {
      o.ls.p.grad(xc, g);
    } else {
      for (int a = 0; a < 3; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < 3; ++b) g[a] += o.ls.q.Q[a][b] * (xc[b] - o.c[b]);
      }
    }
    for (int a = 0; a < 3; ++a) gn += g[a] * g[a];
    gn = std::sqrt(gn);
    for (int a = 0; a < 3; ++a) sgn[a] = (g[a] < -1e-9 * gn) ? -1 : 1;
  }
  std::vector<Numbering> nums[3];
  for (int depth = 0; depth <= 4; ++depth) {
    for (const auto& o : shifts) {
      int lo[3];
      for (int a = 0; a < 3; ++a) lo[a] = std::min(std::max(ii[a] - 2 + sgn[a] * o[a], 0), n - 5);
      bool win[5][5][5];
      for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b)
          for (int c = 0; c < 5; ++c) {
            int q = idx(lo[0] + a, lo[1] + b, lo[2] + c);
            win[a][b][c] = host[q] == q;
          }
      for (int a = 0; a < 3; ++a) axis_numberings(ii[a], lo[a], sgn[a], nums[a]);
      for (const Numbering& nx : nums[0])
        for (const Numbering& ny : nums[1]) {
          int need = depth - nx.k - ny.k;
          if (need < 0) continue;
          for (const Numbering& nz : nums[2]) {
            if (nz.k != need) continue;
            bool ok = true;
            for (int t = 0; t < kPLG && ok; ++t)
              ok = win[nx.pts[T.e4[t][0]] - lo[0]][ny.pts[T.e4[t][1]] - lo[1]][nz.pts[T.e4[t][2]] - lo[2]];
            if (!ok) continue;
            for (int t = 0; t < kPLG; ++t)
              cells[t] = idx(nx.pts[T.e4[t][0]], ny.pts[T.e4[t][1]], nz.pts[T.e4[t][2]]);
            return;
          }
        }
    }
  }
  fail(CC_EPLG, "no poised lattice for cell " + std::to_string(p) + " at n=" + std::to_string(n));
}

// ------------------------------------------------------------- PLG rows
void LevelHost::group_moments(int target, int cell, double out[N4]) const {
  int ti[3];
  ijk(target, ti[0], ti[1], ti[2]);
  std::vector<int> tmp;
  const std::vector<int>& mem = members(cell, tmp);
  double tot[N4] = {}, v = 0.0;
  for (int m : mem) {
    int mi[3];
    ijk(m, mi[0], mi[1], mi[2]);
    int dl[3] = {mi[0] - ti[0], mi[1] - ti[1], mi[2] - ti[2]};
    auto it = cut.find(m);
    const double* mom = (it != cut.end()) ? it->second.m : full_moments().data();
    double sh[N4];
    shift_moments4(mom, dl, sh);
    for (int a = 0; a < N4; ++a) tot[a] += vol[m] * sh[a];
    v += vol[m];
  }
  for (int a = 0; a < N4; ++a) out[a] = tot[a] / v;
}

// min-norm y with M^T y = ell, M (m x 35) row-major, by Householder QR of M.
static bool min_norm_solve(std::vector<double>& M, int m, const double ell[N4], std::vector<double>& y) {
  const int nc = N4;
  std::vector<double> V((size_t)m * nc, 0.0), vv(nc);
  double R[N4][N4];
  double scale = 0.0;
  for (double x : M) scale = std::max(scale, std::fabs(x));
  for (int k = 0; k < nc; ++k) {
    double nrm = 0.0;
    for (int r = k; r < m; ++r) nrm += M[(size_t)r * nc + k] * M[(size_t)r * nc + k];
    nrm = std::sqrt(nrm);
    double x0 = M[(size_t)k * nc + k];
    double alpha = (x0 >= 0) ? -nrm : nrm;
    double vn = 0.0;
    for (int r = k; r < m; ++r) {
      double v = M[(size_t)r * nc + k] - (r == k ? alpha : 0.0);
      V[(size_t)r * nc + k] = v;
      vn += v * v;
    }
    vv[k] = vn;
    if (vn > 0)
      for (int c = k; c < nc; ++c) {
        double dot = 0.0;
        for (int r = k; r < m; ++r) dot += V[(size_t)r * nc + k] * M[(size_t)r * nc + c];
        double f = 2.0 * dot / vn;
        for (int r = k; r < m; ++r) M[(size_t)r * nc + c] -= f * V[(size_t)r * nc + k];
      }
    for (int c = k; c < nc; ++c) R[k][c] = M[(size_t)k * nc + c];
    if (std::fabs(R[k][k]) <= 1e-13 * scale) return false;
  }
  double u[N4];
  for (int k = 0; k < nc; ++k) {
    double s = ell[k];
    for (int i = 0; i < k; ++i) s -= R[i][k] * u[i];
    u[k] = s / R[k][k];
  }
  y.assign(m, 0.0);
  for (int k = 0; k < nc; ++k) y[k] = u[k];
  for (int k = nc - 1; k >= 0; --k) {
    if (vv[k] <= 0) continue;
    double dot = 0.0;
    for (int r = k; r < m; ++r) dot += V[(size_t)r * nc + k] * y[r];
    double f = 2.0 * dot / vv[k];
    for (int r = k; r < m; ++r) y[r] -= f * V[(size_t)r * nc + k];
  }
  return true;
}

void LevelHost::plg_system(int p, int row, const int cells[kPLG], std::vector<double>& M, std::vector<double>& sw,
                           double ell[N4], std::vector<Site>& sites) const {
  const MonoTable& T = mono();
  int ti[3];
  ijk(p, ti[0], ti[1], ti[2]);
  sites.clear();
  std::vector<int> tmp;
  for (int t = 0; t < kPLG; ++t) {
    const std::vector<int>& mem = members(cells[t], tmp);
    for (int m : mem) {
      auto it = cut.find(m);
      if (it != cut.end() && it->second.area > 0)
        sites.push_back({row, 'S', m, dom->obst[it->second.obst].bc, 0, 0, 0.0});
    }
  }
  for (int t = 0; t < kPLG; ++t) {
    int ci[3];
    ijk(cells[t], ci[0], ci[1], ci[2]);
    for (int d = 0; d < 3; ++d)
      for (int side : {-1, 1})
        if ((side < 0 && ci[d] == 0) || (side > 0 && ci[d] == n - 1))
          sites.push_back({row, 'W', cells[t], wall_bc[2 * d + (side > 0 ? 1 : 0)], d, side, 0.0});
  }
  const int m = kPLG + (int)sites.size();
  M.assign((size_t)m * N4, 0.0);
  sw.assign(m, 0.0);
  auto weight = [&](int cell) {
    int ci[3];
    ijk(cell, ci[0], ci[1], ci[2]);
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (double)(ci[a] - ti[a]) * (ci[a] - ti[a]);
    return std::pow(std::max(1.0, d2), -4.0);
  };
  for (int t = 0; t < kPLG; ++t) {
    group_moments(p, cells[t], &M[(size_t)t * N4]);
    sw[t] = std::sqrt(weight(cells[t]));
  }
  for (size_t s = 0; s < sites.size(); ++s) {
    double* rowp = &M[(size_t)(kPLG + s) * N4];
    const Site& st = sites[s];
    int ci[3];
    ijk(st.cell, ci[0], ci[1], ci[2]);
    int dl[3] = {ci[0] - ti[0], ci[1] - ti[1], ci[2] - ti[2]};
    if (st.kind == 'S') {
      const CutData& cd = cut.at(st.cell);
      // Dirichlet: <<xi^a>>; Neumann: <<n . grad_xi xi^a>>; Robin:
      // s (alpha <<xi^a>> + (beta / h) <<n . grad_xi xi^a>>), s = h / (|alpha| h + |beta|)
      double dir[N4], neu[N4];
      if (st.bc != CC_NEUMANN) shift_moments4(cd.sm, dl, dir);
      if (st.bc != CC_DIRICHLET) {
        double sh[3][N3];
        for (int d = 0; d < 3; ++d) shift_moments3(cd.sn[d], dl, sh[d]);
        for (int j = 0; j < N4; ++j) {
          double v = 0.0;
          for (int d = 0; d < 3; ++d) {
            int a[3] = {T.e4[j][0], T.e4[j][1], T.e4[j][2]};
            if (a[d] == 0) continue;
            int e = a[d];
            a[d] -= 1;
            v += e * sh[d][T.idx3[a[0]][a[1]][a[2]]];
          }
          neu[j] = v;
        }
      }
      if (st.bc == CC_DIRICHLET) {
        for (int j = 0; j < N4; ++j) rowp[j] = dir[j];
      } else if (st.bc == CC_NEUMANN) {
        for (int j = 0; j < N4; ++j) rowp[j] = neu[j];
      } else {
        const Obstacle& ob = dom->obst[cd.obst];
        const double sc = h / (std::fabs(ob.alpha) * h + std::fabs(ob.beta));
        for (int j = 0; j < N4; ++j) rowp[j] = sc * (ob.alpha * dir[j] + (ob.beta / h) * neu[j]);
      }
    } else {
      int d = st.axis;
      double xf = dl[d] + 0.5 * st.side;
      for (int j = 0; j < N4; ++j) {
        double inplane = 1.0;
        for (int a = 0; a < 3; ++a)
          if (a != d) {
            int k = T.e4[j][a];
            double dd = dl[a];
            inplane *= (std::pow(dd + 0.5, k + 1) - std::pow(dd - 0.5, k + 1)) / (k + 1);
          }
        int ed = T.e4[j][d];
        const double dir = inplane * ipow(xf, ed);
        const double neu = ed > 0 ? st.side * ed * ipow(xf, ed - 1) * inplane : 0.0;
        if (st.bc == CC_DIRICHLET) {
          rowp[j] = dir;
        } else if (st.bc == CC_NEUMANN) {
          rowp[j] = neu;
        } else {
          // Robin wall: s (alpha <xi^a> + (beta / h) <n . grad_xi xi^a>), s = h / (|alpha| h + |beta|)
          const double* ab = dom->wall_robin[2 * d + (st.side > 0 ? 1 : 0)];
          const double sc = h / (std::fabs(ab[0]) * h + std::fabs(ab[1]));
          rowp[j] = sc * (ab[0] * dir + (ab[1] / h) * neu);
        }
      }
    }
    sw[kPLG + s] = std::sqrt(weight(st.cell));
  }
  for (int r = 0; r < m; ++r)
    for (int j = 0; j < N4; ++j) M[(size_t)r * N4 + j] *= sw[r];
  double mom[N4];
  group_moments(p, p, mom);
  for (int j = 0; j < N4; ++j) {
    double v = 0.0;
    for (int d = 0; d < 3; ++d) {
      int a[3] = {T.e4[j][0], T.e4[j][1], T.e4[j][2]};
      if (a[d] < 2) continue;
      int e = a[d];
      a[d] -= 2;
      v += e * (e - 1) * mom[T.idx4[a[0]][a[1]][a[2]]];
    }
    ell[j] = v / (h * h);
  }
}

void LevelHost::rows(PlgLsqSolver* lsq) {
  const size_t N2 = phi2.size();
  plg_cols.assign(N2 * kPLG, 0);
  plg_vals.assign(N2 * kPLG, 0.0);
  int nt = omp_get_max_threads();
  std::vector<std::vector<Site>> tsites(N2);
  int err_code = 0;
  std::string err_msg;
  auto record = [&](const Error& e) {
#pragma omp critical
    {
      if (!err_code) {
        err_code = e.code;
        err_msg = e.what();
      }
    }
  };
  // the row's value from the fit: c_t = sw_t y_t for the 35 cells, then the sites
  auto finish = [&](long r, const std::vector<double>& sw, const double* y) {
    for (int t = 0; t < kPLG; ++t) plg_vals[(size_t)r * kPLG + t] = sw[t] * y[t];
    for (size_t s = 0; s < tsites[r].size(); ++s) tsites[r][s].coef = sw[kPLG + s] * y[kPLG + s];
  };
  if (!lsq) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (long r = 0; r < (long)N2; ++r) {
      if (err_code) continue;
      try {
        int* cells = &plg_cols[(size_t)r * kPLG];
        plg_select(phi2[r], cells);
        std::vector<double> M, sw, y;
        double ell[N4];
        plg_system(phi2[r], (int)r, cells, M, sw, ell, tsites[r]);
        if (!min_norm_solve(M, (int)sw.size(), ell, y))
          fail(CC_EPLG, "rank-deficient least-squares fit at cell " + std::to_string(phi2[r]));
        finish(r, sw, y.data());
      } catch (const Error& e) {
        record(e);
      }
    }
  } else {
    // the systems in chunks: assembled on the host, solved by lsq (the device)
    const long chunk = 16384;
    std::vector<std::vector<double>> Ms, sws;
    std::vector<double> A, ellv, y;
    std::vector<int> off, ok;
    for (long r0 = 0; r0 < (long)N2 && !err_code; r0 += chunk) {
      const long nr = std::min<long>(chunk, (long)N2 - r0);
      Ms.assign(nr, {});
      sws.assign(nr, {});
      ellv.assign((size_t)nr * N4, 0.0);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
      for (long k = 0; k < nr; ++k) {
        if (err_code) continue;
        const long r = r0 + k;
        try {
          int* cells = &plg_cols[(size_t)r * kPLG];
          plg_select(phi2[r], cells);
          plg_system(phi2[r], (int)r, cells, Ms[k], sws[k], &ellv[(size_t)k * N4], tsites[r]);
        } catch (const Error& e) {
          record(e);
        }
      }
      if (err_code) break;
      off.assign(nr + 1, 0);
      for (long k = 0; k < nr; ++k) off[k + 1] = off[k] + (int)sws[k].size();
      A.assign((size_t)off[nr] * N4, 0.0);
      for (long k = 0; k < nr; ++k) std::copy(Ms[k].begin(), Ms[k].end(), A.begin() + (size_t)off[k] * N4);
      y.assign(off[nr], 0.0);
      ok.assign(nr, 0);
      lsq->solve((int)nr, off.data(), A.data(), ellv.data(), y.data(), ok.data());
      for (long k = 0; k < nr; ++k) {
        if (!ok[k]) fail(CC_EPLG, "rank-deficient least-squares fit at cell " + std::to_string(phi2[r0 + k]));
        finish(r0 + k, sws[k], &y[off[k]]);
      }
    }
  }
  if (err_code) fail(err_code, err_msg);
  sites.clear();
  for (auto& v : tsites) sites.insert(sites.end(), v.begin(), v.end());
}

// Ghost cells beyond a wall, in units of h along its normal (the wall at 0,
// interior cells [j-1, j] with averages A_1..A_4, ghost g = [-g, 1-g]): the
// averages of the quartic P that matches the A_j and the wall condition
// (Dirichlet P(0) = D, Neumann -P'(0)/h = D, Robin alpha P(0) - (beta/h) P'(0) = D).
// G_g = sum_j r_g[j] A_j + r_g[4] D, from M^T r_g = m_g with M the 5 x 5 system
// and m_g the ghost averages of the monomials.  The rows follow by substituting
// G_1, G_2 into the 5-point stencil of the two cells next to the wall.
WallRows wall_rows(int bc, double alpha, double beta, double h) {
  // Dirichlet and Neumann: the exact tables the stencil kernels use
  if (bc == CC_DIRICHLET)
    return WallRows{{{-1087.0 / 12, 545.0 / 12, -139.0 / 12, 21.0 / 12}, {269.0 / 12, -403.0 / 12, 209.0 / 12, -15.0 / 12}},
                    {55.0, -5.0}};
  if (bc == CC_NEUMANN)
    return WallRows{{{-14.5, 15.9, -1.5, 0.1}, {15.5, -30.9, 16.5, -1.1}}, {13.2 * h, -1.2 * h}};
  auto avg = [](int k, double a, double b) { return (std::pow(b, k + 1) - std::pow(a, k + 1)) / ((k + 1) * (b - a)); };
  double r[2][5];
  for (int g = 1; g <= 2; ++g) {
    // solve M^T r = m by Gaussian elimination with partial pivoting (5 x 5)
    double A[5][6];
    for (int k = 0; k < 5; ++k) {       // row k of M^T = column k of M
      for (int j = 0; j < 4; ++j) A[k][j] = avg(k, j, j + 1);
      A[k][4] = (k == 0 ? alpha : 0.0) + (k == 1 ? -beta / h : 0.0);
      A[k][5] = avg(k, -g, 1 - g);
    }
    for (int c = 0; c < 5; ++c) {
      int piv = c;
      for (int q = c + 1; q < 5; ++q)
        if (std::fabs(A[q][c]) > std::fabs(A[piv][c])) piv = q;
      if (piv != c)
        for (int t = 0; t < 6; ++t) std::swap(A[c][t], A[piv][t]);
      for (int q = c + 1; q < 5; ++q) {
        const double f = A[q][c] / A[c][c];
        for (int t = c; t < 6; ++t) A[q][t] -= f * A[c][t];
      }
    }
    for (int c = 4; c >= 0; --c) {
      double v = A[c][5];
      for (int t = c + 1; t < 5; ++t) v -= A[c][t] * r[g - 1][t];
      r[g - 1][c] = v / A[c][c];
    }
  }
  WallRows w;
  // layer 0: -G_2 + 16 G_1 - 30 A_1 + 16 A_2 - A_3
  const double base0[4] = {-30.0, 16.0, -1.0, 0.0};
  for (int j = 0; j < 4; ++j) w.lay[0][j] = base0[j] + 16.0 * r[0][j] - r[1][j];
  w.dat[0] = 16.0 * r[0][4] - r[1][4];
  // layer 1: -G_1 + 16 A_1 - 30 A_2 + 16 A_3 - A_4
  const double base1[4] = {16.0, -30.0, 16.0, -1.0};
  for (int j = 0; j < 4; ++j) w.lay[1][j] = base1[j] - r[0][j];
  w.dat[1] = -r[0][4];
  return w;
}

}  // namespace cc
