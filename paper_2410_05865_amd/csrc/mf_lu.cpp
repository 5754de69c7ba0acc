// Nested dissection + multifrontal LU; see mf_lu.hpp.
#include "mf_lu.hpp"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>
#include <string>
#include <unordered_map>

#include "common.hpp"

namespace cc {

namespace {

struct TNode {
  std::vector<int> F;   // original vertex ids
  int left = -1, right = -1;
};

struct Builder {
  const std::vector<std::vector<int>>* adj;
  const std::vector<std::array<int, 3>>* xyz;
  int leaf;
  std::vector<TNode> t;
  std::vector<int> mark;   // scratch: side of each vertex during a split

  // Connected components of verts (in the graph restricted to verts), largest
  // first; mark[] is left zero.
  std::vector<std::vector<int>> components(const std::vector<int>& verts) {
    for (int v : verts) mark[v] = 1;
    std::vector<std::vector<int>> comps;
    std::vector<int> stack;
    for (int v0 : verts) {
      if (mark[v0] != 1) continue;
      comps.emplace_back();
      std::vector<int>& c = comps.back();
      mark[v0] = 2;
      stack.push_back(v0);
      while (!stack.empty()) {
        int v = stack.back();
        stack.pop_back();
        c.push_back(v);
        for (int w : (*adj)[v])
          if (mark[w] == 1) {
            mark[w] = 2;
            stack.push_back(w);
          }
      }
    }
    for (int v : verts) mark[v] = 0;
    std::stable_sort(comps.begin(), comps.end(),
                     [](const std::vector<int>& a, const std::vector<int>& b) { return a.size() > b.size(); });
    return comps;
  }

  int build(std::vector<int>& verts) {
    int id = (int)t.size();
    t.emplace_back();
    if ((int)verts.size() <= leaf) {
      std::sort(verts.begin(), verts.end());
      t[id].F = verts;
      return id;
    }
    // Disconnected vertex sets need no separator: split the components into
    // two groups of similar size under an empty node.
    {
      std::vector<std::vector<int>> comps = components(verts);
      if (comps.size() > 1) {
        std::vector<int> L, R;
        for (auto& c : comps) {
          std::vector<int>& dst = L.size() <= R.size() ? L : R;
          dst.insert(dst.end(), c.begin(), c.end());
        }
        int l = build(L);
        t[id].left = l;
        int r = build(R);
        t[id].right = r;
        return id;
      }
    }
    // Candidate cuts: a few planes per axis (quantiles of the coordinates);
    // for each, the vertex separator is the smaller of the two one-sided sets
    // (vertices of one side adjacent to the other).  The smallest separator
    // with both halves holding at least 30% of the rest wins; ties keep the
    // earlier candidate (largest-extent axis first, median first).
    int order[3] = {0, 1, 2};
    int ext[3];
    for (int a = 0; a < 3; ++a) {
      int lo = INT32_MAX, hi = INT32_MIN;
      for (int v : verts) {
        lo = std::min(lo, (*xyz)[v][a]);
        hi = std::max(hi, (*xyz)[v][a]);
      }
      ext[a] = hi - lo;
    }
    std::stable_sort(order, order + 3, [&](int x, int y) { return ext[x] > ext[y]; });
    if (ext[order[0]] == 0) {
      std::sort(verts.begin(), verts.end());
      t[id].F = verts;
      return id;
    }
    static const double kQuant[5] = {0.5, 0.42, 0.58, 0.35, 0.65};
    const size_t nv = verts.size();
    size_t best_size = SIZE_MAX;
    int best_axis = -1, best_c = 0, best_side = 1;
    std::vector<int> cs(nv);
    for (int oa = 0; oa < 3; ++oa) {
      int axis = order[oa];
      if (ext[axis] == 0) continue;
      for (size_t i = 0; i < nv; ++i) cs[i] = (*xyz)[verts[i]][axis];
      std::sort(cs.begin(), cs.end());
      int nq = (oa == 0) ? 5 : 1;
      for (int qi = 0; qi < nq; ++qi) {
        int c = cs[std::min(nv - 1, (size_t)(kQuant[qi] * nv))];
        if (c == cs[0]) {
          auto it = std::upper_bound(cs.begin(), cs.end(), cs[0]);
          if (it == cs.end()) continue;
          c = *it;
        }
        for (int v : verts) mark[v] = ((*xyz)[v][axis] < c) ? 1 : 2;
        size_t nl = 0, sl = 0, sr = 0;
        for (int v : verts) {
          bool left = mark[v] == 1;
          nl += left;
          for (int w : (*adj)[v])
            if (mark[w] != 0 && mark[w] != mark[v]) {
              (left ? sl : sr)++;
              break;
            }
        }
        for (int v : verts) mark[v] = 0;
        size_t nr = nv - nl;
        for (int side = 1; side <= 2; ++side) {
          size_t sep = side == 1 ? sl : sr;
          size_t a = (side == 1 ? nl : nr) - sep, b = (side == 1 ? nr : nl);
          size_t rest = a + b;
          if (rest == 0) continue;
          bool balanced = a >= 0.3 * rest && b >= 0.3 * rest;
          if (!balanced && !(best_axis < 0 && qi == 0 && oa == 0)) continue;
          if (sep < best_size) {
            best_size = sep;
            best_axis = axis;
            best_c = c;
            best_side = side;
          }
        }
      }
    }
    if (best_axis < 0) {
      std::sort(verts.begin(), verts.end());
      t[id].F = verts;
      return id;
    }
    for (int v : verts) mark[v] = ((*xyz)[v][best_axis] < best_c) ? 1 : 2;
    std::vector<int> L, R, S;
    for (int v : verts) {
      bool mine = mark[v] == best_side;
      bool touches = false;
      if (mine)
        for (int w : (*adj)[v])
          if (mark[w] != 0 && mark[w] != mark[v]) {
            touches = true;
            break;
          }
      if (touches)
        S.push_back(v);
      else
        (mark[v] == 1 ? L : R).push_back(v);
    }
    for (int v : verts) mark[v] = 0;
    std::sort(S.begin(), S.end());
    t[id].F = S;
    if (!L.empty()) {
      int l = build(L);
      t[id].left = l;
    }
    if (!R.empty()) {
      int r = build(R);
      t[id].right = r;
    }
    return id;
  }
};

// Blocked right-looking LU of the leading p columns of the f x f row-major front,
// pivoting among rows [k, p).  rowperm receives the final order of rows 0..p-1.
void front_lu(std::vector<double>& A, int f, int p, std::vector<int>& rowperm, double tiny, bool par) {
  rowperm.resize(p);
  std::iota(rowperm.begin(), rowperm.end(), 0);
  const int nb = 48;
  for (int k0 = 0; k0 < p; k0 += nb) {
    int kb = std::min(nb, p - k0);
    int kend = k0 + kb;
    for (int k = k0; k < kend; ++k) {
      int piv = k;
      double best = std::fabs(A[(size_t)k * f + k]);
      for (int r = k + 1; r < p; ++r) {
        double v = std::fabs(A[(size_t)r * f + k]);
        if (v > best) {
          best = v;
          piv = r;
        }
      }
      if (!(best > tiny)) fail(CC_ESINGULAR, "pivot below threshold in a front");
      if (piv != k) {
        std::swap_ranges(A.begin() + (size_t)k * f, A.begin() + (size_t)k * f + f, A.begin() + (size_t)piv * f);
        std::swap(rowperm[k], rowperm[piv]);
      }
      double d = A[(size_t)k * f + k];
      const double* rk = &A[(size_t)k * f];
#pragma omp parallel for schedule(static) if (par && f - k > 256)
      for (int r = k + 1; r < f; ++r) {
        double* rr = &A[(size_t)r * f];
        double l = rr[k] / d;
        rr[k] = l;
        for (int c = k + 1; c < kend; ++c) rr[c] -= l * rk[c];
      }
    }
    if (kend >= f) continue;
    // block row U12 = L_panel^-1 A[k0:kend, kend:]
    for (int k = k0; k < kend; ++k) {
      const double* rk = &A[(size_t)k * f];
      for (int r = k + 1; r < kend; ++r) {
        double* rr = &A[(size_t)r * f];
        double l = rr[k];
        for (int c = kend; c < f; ++c) rr[c] -= l * rk[c];
      }
    }
    // trailing update
#pragma omp parallel for schedule(dynamic, 8) if (par && f - kend > 128)
    for (int r = kend; r < f; ++r) {
      double* rr = &A[(size_t)r * f];
      for (int k = k0; k < kend; ++k) {
        double l = rr[k];
        if (l == 0.0) continue;
        const double* rk = &A[(size_t)k * f];
        for (int c = kend; c < f; ++c) rr[c] -= l * rk[c];
      }
    }
  }
}

}  // namespace

void factorize(const CSR& A, const std::vector<std::array<int, 3>>& coords, int leaf, double pivot_tol,
               SupernodalLU& out) {
  const int n = A.n;
  out = SupernodalLU();
  out.n = n;
  if (n == 0) return;
  // symmetrised adjacency (no diagonal)
  std::vector<std::vector<int>> adj(n);
  double amax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      int j = A.col[e];
      amax = std::max(amax, std::fabs(A.val[e]));
      if (j == i) continue;
      adj[i].push_back(j);
      adj[j].push_back(i);
    }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  Builder B;
  B.adj = &adj;
  B.xyz = &coords;
  B.leaf = std::max(1, leaf);
  B.mark.assign(n, 0);
  std::vector<int> all(n);
  std::iota(all.begin(), all.end(), 0);
  int root = B.build(all);
  // postorder
  std::vector<int> post;
  std::vector<int> tparent(B.t.size(), -1);
  {
    std::vector<std::pair<int, int>> st = {{root, 0}};
    while (!st.empty()) {
      auto& [id, state] = st.back();
      if (state == 0) {
        state = 1;
        if (B.t[id].left >= 0) {
          tparent[B.t[id].left] = id;
          st.push_back({B.t[id].left, 0});
        }
      } else if (state == 1) {
        state = 2;
        if (B.t[id].right >= 0) {
          tparent[B.t[id].right] = id;
          st.push_back({B.t[id].right, 0});
        }
      } else {
        post.push_back(id);
        st.pop_back();
      }
    }
  }
  // drop empty separators: their children attach to the nearest non-empty ancestor
  std::vector<int> tnode_to_sn(B.t.size(), -1);
  out.perm.assign(n, -1);
  out.iperm.assign(n, -1);
  int next = 0;
  for (int id : post) {
    if (B.t[id].F.empty()) continue;
    SnNode nd;
    nd.base = next;
    nd.p = (int)B.t[id].F.size();
    for (int v : B.t[id].F) {
      out.perm[next] = v;
      out.iperm[v] = next;
      ++next;
    }
    tnode_to_sn[id] = (int)out.nodes.size();
    out.nodes.push_back(nd);
  }
  if (next != n) fail(CC_EINVAL, "nested dissection lost vertices");
  const int ns = (int)out.nodes.size();
  for (int id : post) {
    int s = tnode_to_sn[id];
    if (s < 0) continue;
    int a = tparent[id];
    while (a >= 0 && tnode_to_sn[a] < 0) a = tparent[a];
    out.nodes[s].parent = (a >= 0) ? tnode_to_sn[a] : -1;
  }
  // subtree index ranges for the separator check
  std::vector<int> lo_idx(ns);
  for (int s = 0; s < ns; ++s) lo_idx[s] = out.nodes[s].base;
  for (int s = 0; s < ns; ++s) {
    int pa = out.nodes[s].parent;
    if (pa >= 0) lo_idx[pa] = std::min(lo_idx[pa], lo_idx[s]);
  }
  std::vector<int> node_of(n);
  for (int s = 0; s < ns; ++s)
    for (int v = out.nodes[s].base; v < out.nodes[s].base + out.nodes[s].p; ++v) node_of[v] = s;
  // symbolic: U sets
  std::vector<std::vector<int>> U(ns);
  std::vector<std::vector<int>> children(ns);
  for (int s = 0; s < ns; ++s)
    if (out.nodes[s].parent >= 0) children[out.nodes[s].parent].push_back(s);
  for (int s = 0; s < ns; ++s) {
    const SnNode& nd = out.nodes[s];
    int last = nd.base + nd.p - 1;
    std::vector<int> u;
    for (int v = nd.base; v <= last; ++v)
      for (int w0 : adj[out.perm[v]]) {
        int w = out.iperm[w0];
        if (w > last) u.push_back(w);
      }
    for (int c : children[s])
      for (int w : U[c])
        if (w > last) u.push_back(w);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (int w : u) {
      int a = node_of[w];
      if (!(lo_idx[a] <= nd.base && nd.base + nd.p - 1 <= out.nodes[a].base + out.nodes[a].p - 1))
        fail(CC_EINVAL, "nested dissection separator check failed");
    }
    U[s] = std::move(u);
  }
  // heights
  for (int s = 0; s < ns; ++s) {
    int pa = out.nodes[s].parent;
    if (pa >= 0) out.nodes[pa].height = std::max(out.nodes[pa].height, out.nodes[s].height + 1);
  }
  for (const SnNode& nd : out.nodes) out.max_height = std::max(out.max_height, nd.height);
  // storage offsets
  long long oM = 0, oV = 0, oW = 0, oU = 0, oP = 0;
  for (int s = 0; s < ns; ++s) {
    SnNode& nd = out.nodes[s];
    nd.q = (int)U[s].size();
    nd.offM = oM;
    nd.offV = oV;
    nd.offW = oW;
    nd.offU = oU;
    nd.offPiv = oP;
    oM += (long long)nd.p * nd.p;
    oV += (long long)nd.q * nd.p;
    oW += (long long)nd.p * nd.q;
    oU += nd.q;
    oP += nd.p;
  }
  out.Mbuf.assign(oM, 0.0);
  out.Vbuf.assign(oV, 0.0);
  out.Wbuf.assign(oW, 0.0);
  out.Ubuf.assign(oU, 0);
  out.Pivbuf.assign(oP, 0);
  for (int s = 0; s < ns; ++s) std::copy(U[s].begin(), U[s].end(), out.Ubuf.begin() + out.nodes[s].offU);
  // transpose pattern for column assembly
  std::vector<int> tptr(n + 1, 0), trow(A.ptr[n]);
  std::vector<double> tval(A.ptr[n]);
  for (int e = 0; e < A.ptr[n]; ++e) tptr[A.col[e] + 1]++;
  for (int i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  {
    std::vector<int> fill(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        int c = A.col[e];
        trow[fill[c]] = i;
        tval[fill[c]] = A.val[e];
        fill[c]++;
      }
  }
  const double tiny = pivot_tol * amax;
  std::vector<std::vector<double>> schur(ns);
  // numeric factorisation, by height (nodes of one height are independent)
  std::vector<std::vector<int>> by_h(out.max_height + 1);
  for (int s = 0; s < ns; ++s) by_h[out.nodes[s].height].push_back(s);
  int err_code = 0;
  std::string err_msg;
  for (int hgt = 0; hgt <= out.max_height; ++hgt) {
    const std::vector<int>& lst = by_h[hgt];
    auto work = [&](int s, bool par) {
      const SnNode& nd = out.nodes[s];
      const int p = nd.p, q = nd.q, f = p + q;
      const std::vector<int>& Us = U[s];
      auto loc = [&](int w) -> int {
        if (w >= nd.base && w < nd.base + p) return w - nd.base;
        auto it = std::lower_bound(Us.begin(), Us.end(), w);
        if (it == Us.end() || *it != w) return -1;
        return p + (int)(it - Us.begin());
      };
      std::vector<double> Fm((size_t)f * f, 0.0);
      for (int v = nd.base; v < nd.base + p; ++v) {
        int ov = out.perm[v];
        int lv = v - nd.base;
        for (int e = A.ptr[ov]; e < A.ptr[ov + 1]; ++e) {
          int w = out.iperm[A.col[e]];
          if (w < nd.base) continue;
          int lw = loc(w);
          if (lw < 0) fail(CC_EINVAL, "front assembly: column outside the front");
          Fm[(size_t)lv * f + lw] += A.val[e];
        }
        for (int e = tptr[ov]; e < tptr[ov + 1]; ++e) {
          int w = out.iperm[trow[e]];
          if (w < nd.base + p) continue;
          int lw = loc(w);
          if (lw < 0) fail(CC_EINVAL, "front assembly: row outside the front");
          Fm[(size_t)lw * f + lv] += tval[e];
        }
      }
      for (int c : children[s]) {
        const std::vector<int>& Uc = U[c];
        const std::vector<double>& S = schur[c];
        int qc = (int)Uc.size();
        std::vector<int> lc(qc);
        for (int i = 0; i < qc; ++i) {
          lc[i] = loc(Uc[i]);
          if (lc[i] < 0) fail(CC_EINVAL, "extend-add outside the parent front");
        }
        for (int i = 0; i < qc; ++i)
          for (int j = 0; j < qc; ++j) Fm[(size_t)lc[i] * f + lc[j]] += S[(size_t)i * qc + j];
      }
      for (int c : children[s]) std::vector<double>().swap(schur[c]);
      std::vector<int> rowperm;
      front_lu(Fm, f, p, rowperm, tiny, par);
      for (int j = 0; j < p; ++j) out.Pivbuf[nd.offPiv + j] = rowperm[j];
      // inverses of L11 (unit lower) and U11 into M
      double* M = &out.Mbuf[nd.offM];
      std::vector<double> iL((size_t)p * p, 0.0), iU((size_t)p * p, 0.0);
#pragma omp parallel for schedule(dynamic, 16) if (par && p > 128)
      for (int c = 0; c < p; ++c) {
        // column c of L11^-1: forward substitution with e_c
        iL[(size_t)c * p + c] = 1.0;
        for (int r = c + 1; r < p; ++r) {
          double s2 = 0.0;
          for (int k = c; k < r; ++k) s2 += Fm[(size_t)r * f + k] * iL[(size_t)k * p + c];
          iL[(size_t)r * p + c] = -s2;
        }
        // column c of U11^-1: back substitution with e_c
        for (int r = c; r >= 0; --r) {
          double s2 = (r == c) ? 1.0 : 0.0;
          for (int k = r + 1; k <= c; ++k) s2 -= Fm[(size_t)r * f + k] * iU[(size_t)k * p + c];
          iU[(size_t)r * p + c] = s2 / Fm[(size_t)r * f + r];
        }
      }
      for (int r = 0; r < p; ++r)
        for (int c = 0; c < p; ++c) M[(size_t)r * p + c] = (c < r) ? iL[(size_t)r * p + c] : iU[(size_t)r * p + c];
      if (q > 0) {
        double* V = &out.Vbuf[nd.offV];
        double* W = &out.Wbuf[nd.offW];
        // V = L21 iL  (q x p)
#pragma omp parallel for schedule(static) if (par && q > 64)
        for (int r = 0; r < q; ++r) {
          const double* l21 = &Fm[(size_t)(p + r) * f];
          double* vr = V + (size_t)r * p;
          for (int k = 0; k < p; ++k) {
            double a = l21[k];
            if (a == 0.0) continue;
            const double* il = &iL[(size_t)k * p];
            for (int c = 0; c <= k; ++c) vr[c] += a * il[c];
          }
        }
        // W = iU U12  (p x q)
#pragma omp parallel for schedule(static) if (par && p > 64)
        for (int r = 0; r < p; ++r) {
          double* wr = W + (size_t)r * q;
          for (int k = r; k < p; ++k) {
            double a = iU[(size_t)r * p + k];
            if (a == 0.0) continue;
            const double* u12 = &Fm[(size_t)k * f + p];
            for (int c = 0; c < q; ++c) wr[c] += a * u12[c];
          }
        }
        std::vector<double> S((size_t)q * q);
        for (int r = 0; r < q; ++r)
          std::copy(Fm.begin() + (size_t)(p + r) * f + p, Fm.begin() + (size_t)(p + r) * f + f,
                    S.begin() + (size_t)r * q);
        schur[s] = std::move(S);
      }
    };
    bool small = true;
    for (int s : lst) small = small && (out.nodes[s].p + out.nodes[s].q) < 512;
    if (small && lst.size() > 1) {
#pragma omp parallel for schedule(dynamic, 1)
      for (long t = 0; t < (long)lst.size(); ++t) {
        if (err_code) continue;
        try {
          work(lst[t], false);
        } catch (const Error& e) {
#pragma omp critical
          {
            if (!err_code) {
              err_code = e.code;
              err_msg = e.what();
            }
          }
        }
      }
      if (err_code) fail(err_code, err_msg);
    } else {
      for (int s : lst) work(s, true);
    }
  }
}

double selfcheck(const CSR& A, const SupernodalLU& F, unsigned seed) {
  const int n = F.n;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> b(n), y(n), z(n, 0.0), x(n, 0.0);
  for (int i = 0; i < n; ++i) b[i] = U(rng);
  // y in ND order
  for (int v = 0; v < n; ++v) y[v] = b[F.perm[v]];
  std::vector<std::vector<int>> by_h(F.max_height + 1);
  for (int s = 0; s < (int)F.nodes.size(); ++s) by_h[F.nodes[s].height].push_back(s);
  for (int hgt = 0; hgt <= F.max_height; ++hgt) {
    std::vector<std::pair<int, double>> upd;
    for (int s : by_h[hgt]) {
      const SnNode& nd = F.nodes[s];
      std::vector<double> yh(nd.p);
      for (int j = 0; j < nd.p; ++j) yh[j] = y[nd.base + F.Pivbuf[nd.offPiv + j]];
      const double* M = &F.Mbuf[nd.offM];
      for (int r = 0; r < nd.p; ++r) {
        double s2 = yh[r];
        for (int j = 0; j < r; ++j) s2 += M[(size_t)r * nd.p + j] * yh[j];
        z[nd.base + r] = s2;
      }
      for (int r = 0; r < nd.q; ++r) {
        double s2 = 0.0;
        for (int j = 0; j < nd.p; ++j) s2 += F.Vbuf[nd.offV + (size_t)r * nd.p + j] * yh[j];
        upd.push_back({F.Ubuf[nd.offU + r], s2});
      }
    }
    for (auto& u : upd) y[u.first] -= u.second;
  }
  for (int hgt = F.max_height; hgt >= 0; --hgt)
    for (int s : by_h[hgt]) {
      const SnNode& nd = F.nodes[s];
      const double* M = &F.Mbuf[nd.offM];
      for (int r = 0; r < nd.p; ++r) {
        double s2 = 0.0;
        for (int j = r; j < nd.p; ++j) s2 += M[(size_t)r * nd.p + j] * z[nd.base + j];
        for (int j = 0; j < nd.q; ++j) s2 -= F.Wbuf[nd.offW + (size_t)r * nd.q + j] * x[F.Ubuf[nd.offU + j]];
        x[nd.base + r] = s2;
      }
    }
  std::vector<double> xo(n);
  for (int v = 0; v < n; ++v) xo[F.perm[v]] = x[v];
  double rmax = 0.0, bmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double s2 = b[i];
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) s2 -= A.val[e] * xo[A.col[e]];
    rmax = std::max(rmax, std::fabs(s2));
    bmax = std::max(bmax, std::fabs(b[i]));
  }
  return rmax / bmax;
}

}  // namespace cc
