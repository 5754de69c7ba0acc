// C ABI of the solver (include/cutcell.h): build, right-hand side, multigrid
// solve and per-step hooks.  Orchestrates the host setup (level.cpp, mf_lu.cpp)
// and the device kernels (kernels.hip) on one HIP stream.
#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "level.hpp"
#include "mf_lu.hpp"
#include "quadrature.hpp"

namespace cc {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

#define HIPCHK(expr)                                                                                \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess) fail(CC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));      \
  } while (0)
// Synchronize a stream and report launch errors with it: a kernel launch that
// fails (invalid configuration, no code object for the device) has no status
// of its own and shows only in hipGetLastError.
#define HIPSYNC(st)                      \
  do {                                   \
    HIPCHK(hipGetLastError());           \
    HIPCHK(hipStreamSynchronize(st));    \
  } while (0)

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Regular-row entries of a phi_1 cell (coefficients times 12 h^2), same tables
// as the device stencil; Robin walls take the level's assembled wall rows.
void regular_entries(int n, const int bc[6], const WallRows wr[6], int i, int j, int k, std::map<int, double>& row) {
  int ii[3] = {i, j, k};
  long stride[3] = {1, n, (long)n * n};
  long c = i + (long)n * (j + (long)n * k);
  for (int d = 0; d < 3; ++d) {
    int t = ii[d];
    long s = stride[d];
    int blo = bc[2 * d], bhi = bc[2 * d + 1];
    auto add = [&](long off, double v) { row[(int)(c + off * s)] += v; };
    if (t >= 2 && t <= n - 3) {
      add(-2, -1.0); add(-1, 16.0); add(0, -30.0); add(1, 16.0); add(2, -1.0);
    } else if (t == n - 1) {
      if (bhi == CC_ROBIN) { for (int q = 0; q < 4; ++q) add(-q, wr[2 * d + 1].lay[0][q]); }
      else if (bhi == 0) { add(-3, 21.0 / 12); add(-2, -139.0 / 12); add(-1, 545.0 / 12); add(0, -1087.0 / 12); }
      else { add(-3, 0.1); add(-2, -1.5); add(-1, 15.9); add(0, -14.5); }
    } else if (t == n - 2) {
      if (bhi == CC_ROBIN) { for (int q = 0; q < 4; ++q) add(1 - q, wr[2 * d + 1].lay[1][q]); }
      else if (bhi == 0) { add(-2, -15.0 / 12); add(-1, 209.0 / 12); add(0, -403.0 / 12); add(1, 269.0 / 12); }
      else { add(-2, -1.1); add(-1, 16.5); add(0, -30.9); add(1, 15.5); }
    } else if (t == 0) {
      if (blo == CC_ROBIN) { for (int q = 0; q < 4; ++q) add(q, wr[2 * d].lay[0][q]); }
      else if (blo == 0) { add(3, 21.0 / 12); add(2, -139.0 / 12); add(1, 545.0 / 12); add(0, -1087.0 / 12); }
      else { add(3, 0.1); add(2, -1.5); add(1, 15.9); add(0, -14.5); }
    } else {  // t == 1
      if (blo == CC_ROBIN) { for (int q = 0; q < 4; ++q) add(q - 1, wr[2 * d].lay[1][q]); }
      else if (blo == 0) { add(2, -15.0 / 12); add(1, 209.0 / 12); add(0, -403.0 / 12); add(-1, 269.0 / 12); }
      else { add(2, -1.1); add(1, 16.5); add(0, -30.9); add(-1, 15.5); }
    }
  }
}

struct DevBuf {
  std::vector<void*> ptrs;
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) fail(CC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(p);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
  // free one allocation of this buffer (no-op for null)
  void free(void* p) {
    if (!p) return;
    for (size_t i = 0; i < ptrs.size(); ++i)
      if (ptrs[i] == p) {
        (void)hipFree(p);
        ptrs.erase(ptrs.begin() + (long)i);
        return;
      }
  }
};

// Device allocations freed when the scope ends (hipFree waits for the device).
struct TempBuf : DevBuf {
  TempBuf() = default;
  TempBuf(const TempBuf&) = delete;
  TempBuf& operator=(const TempBuf&) = delete;
  ~TempBuf() { release(); }
};

struct DevLU {
  LuDev d{};
  std::vector<LuTasks> tasks;  // per height, all nodes
  LuSub sub;                   // the heights below sub.hcut grouped in subtrees
  bool sub_on = false;         // sweeps use the subtrees (chosen by timing at build)
  double epl = 8.0;            // factor entries per lane of the task lists (chosen by timing)
  int height = 0;
  float tune_ms[10] = {};      // build-time trials: ms per solve, [2k + subtree on] for 2^(k+1) entries
  int wcap = 1 << 30;          // single RHS: wavefronts per height launch at most (chosen by timing)
  LuFlow flow;                 // the one-launch sweeps of a single right-hand side
  bool flow_on = false;        // single-RHS solves use them (cc_set_lu_schedule)
};

// One LU solve with a level's factorization: forward then backward sweeps,
// through the subtree launch for the low heights if chosen, one launch per
// height above; the backward sweep writes the solution to `out`.
template <class T, class TO>
void lu_sweeps(hipStream_t st, const DevLU& L, const LuDev& F, TO* out, long long ostride, int nb) {
  if (L.flow_on && nb == 1) {
    launch_lu_flow<T, TO>(F, L.flow, out, st);
    return;
  }
  const int h0 = L.sub_on ? L.sub.hcut : 0;
  if (L.sub_on) launch_lu_forward_sub<T>(F, L.sub, nb, st);
  for (int h = h0; h <= L.height; ++h) launch_lu_forward<T>(F, L.tasks[h], nb, st);
  for (int h = L.height; h >= h0; --h) launch_lu_backward<T, TO>(F, L.tasks[h], out, ostride, nb, st);
  if (L.sub_on) launch_lu_backward_sub<T, TO>(F, L.sub, out, ostride, nb, st);
}

constexpr int kStencilTrials = 9;  // one cell per thread; marching with 4, 8, 16, 32 planes, in the
                                   // launch order and in the XCD-aware tile order

struct DevLevel {
  StencilLevel st{};
  float stencil_tune_us[kStencilTrials] = {};  // build-time trials: us per FP64 SMO-1 sweep
  int tuned_march = 0, tuned_kz = 8;           // the schedule the trials chose
  int* near = nullptr;                         // phi_1 cells of zone 1 (the near SMO-1 sweep)
  int n_near = 0;
  PlgRows plg{};
  DevLU lu;
  DevBuf sched;  // device task lists of lu's current schedule
  double* s = nullptr;
  double* e = nullptr;
  double* et = nullptr;
  int2* absorbed = nullptr;
  int n_absorbed = 0;
};

inline long long cube(int n) { return (long long)n * n * n; }

// Arrays of the V-cycle in working precision T for nb right-hand sides: per
// level s, e, et (nb * n^3 each), factorization work vectors (nb per variable;
// FP64 on the coarsest level), the FP64 outer residual and per-RHS norms, and
// the captured outer iteration.
template <class T>
struct Work {
  int nb = 0;
  std::vector<T*> s, e, et;
  std::vector<LuDev> lu;
  double* s0 = nullptr;
  unsigned long long* norm = nullptr;
  DevBuf own;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const double* g_r = nullptr;
  double* g_phi = nullptr;
  int g_nb = 0;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    g_r = nullptr;
    g_phi = nullptr;
    g_nb = 0;
  }
  void release() {
    drop_graph();
    own.release();
    s.clear();
    e.clear();
    et.clear();
    lu.clear();
    nb = 0;
  }
};

// Restarted GMRES workspace: k+1 Arnoldi vectors, k preconditioned vectors,
// one work vector (all level-0 grids), small device buffers.
struct Krylov {
  int k = 0;
  DevBuf own;
  double* V = nullptr;
  double* Z = nullptr;
  double* w = nullptr;
  double* d = nullptr;
  unsigned long long* amax = nullptr;
};

}  // namespace

}  // namespace cc

struct cc_problem {
  cc::DomainSpec dom;
  cc_params prm{};
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<std::unique_ptr<cc::LevelHost>> lv;
  std::vector<cc::SupernodalLU> lu;
  std::vector<cc::CSR> lu_mat;
  std::vector<double> setup_s;
  std::vector<double> lu_s;     // per level: the factorization's share of setup_s
  std::vector<cc::DevLevel> dev;
  cc::DevBuf buf;
  unsigned long long* d_norm = nullptr;
  double* d_partial = nullptr;  // reduction scratch (kReductionScratch doubles)
  double* s0 = nullptr;
  double* e0 = nullptr;
  cc::Work<double> w64;         // FP64, one right-hand side (arrays of dev[])
  cc::Work<float> w32;          // mixed precision, one right-hand side
  cc::Work<double> wb64;        // batched
  cc::Work<float> wb32;
  std::vector<float*> volfrac;  // learned guess: per-level volume fractions (uploaded on demand)
  unsigned long long* pair_norm = nullptr;  // training pairs: max|r| of each right-hand side of a group
  float* net_x = nullptr;
  float* net_y = nullptr;
  long long net_cells = 0;
  cc::Krylov kr;                // GMRES acceleration (cc_params.krylov > 0)
  hipStream_t stream2 = nullptr;  // side stream: the far SMO-1 sweeps beside the LU-correction
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int overlap = 0;              // split SMO-1 into far and near sweeps around each SMO-2 (off by
                                // default: measured slower at 256^3, 131.0 against 121.2 ms)
  std::vector<double*> fmg_rhs;  // full multigrid: right-hand side and solution of levels 1..M
  std::vector<double*> fmg_x;    // (allocated on the first cc_fmg, for fmg_nb arrays)
  int fmg_nb = 0;
};

namespace cc {
namespace {

void check_level(const cc_problem* p, int level) {
  if (!p) fail(CC_EINVAL, "null problem");
  if (level < 0 || level >= (int)p->lv.size()) fail(CC_EINVAL, "level out of range");
}
void need_device(const cc_problem* p) {
  if (p->device < 0) fail(CC_EDEVICE, "host-only problem handle (built with device = -1)");
}

// ---------------------------------------------------------------- build
void build_lu_matrix(const LevelHost& L, bool bottom, CSR& A, std::vector<std::array<int, 3>>& xyz,
                     std::vector<int>& var_cell_orig) {
  const int n = L.n;
  std::vector<int> idx_of(L.type.size(), -1);
  const std::vector<int>& vars = bottom ? L.unknowns : L.phi2;
  for (size_t t = 0; t < vars.size(); ++t) idx_of[vars[t]] = (int)t;
  std::vector<int> plg_row(L.type.size(), -1);
  for (size_t r = 0; r < L.phi2.size(); ++r) plg_row[L.phi2[r]] = (int)r;
  A.n = (int)vars.size();
  A.ptr.assign(A.n + 1, 0);
  A.col.clear();
  A.val.clear();
  xyz.resize(A.n);
  var_cell_orig = vars;
  const double s12 = 1.0 / (12.0 * L.h * L.h);
  for (int t = 0; t < A.n; ++t) {
    int c = vars[t];
    int i, j, k;
    L.ijk(c, i, j, k);
    xyz[t] = {i, j, k};
    std::map<int, double> row;
    if (L.type[c] == kPhi1) {
      regular_entries(n, L.wall_bc, L.wall, i, j, k, row);
      for (auto& kv : row) kv.second *= s12;
    } else {
      int r = plg_row[c];
      for (int q = 0; q < kPLG; ++q) row[L.plg_cols[(size_t)r * kPLG + q]] += L.plg_vals[(size_t)r * kPLG + q];
    }
    for (auto& kv : row) {
      int col = idx_of[kv.first];
      if (col < 0) {
        if (bottom) fail(CC_EINVAL, "bottom row references a cell without an unknown");
        continue;  // L21 entry
      }
      A.col.push_back(col);
      A.val.push_back(kv.second);
    }
    A.ptr[t + 1] = (int)A.col.size();
  }
}

// Device copy of a factorization.  Equations of each node are stored in its
// pivot order: position base + j holds equation base + piv[j]; row_pos maps an
// equation (ND index) to its position.
void upload_lu(cc_problem* P, const SupernodalLU& F, const std::vector<int>& var_orig_cell, bool fp32, DevLU& D,
               std::vector<int>& row_pos) {
  DevBuf& B = P->buf;
  const int ns = (int)F.nodes.size();
  std::vector<int> var_cell(F.n), row_cell(F.n);
  for (int v = 0; v < F.n; ++v) var_cell[v] = var_orig_cell[F.perm[v]];
  row_pos.assign(F.n, 0);
  for (int s = 0; s < ns; ++s) {
    const SnNode& nd = F.nodes[s];
    for (int j = 0; j < nd.p; ++j) {
      int eq = nd.base + F.Pivbuf[nd.offPiv + j];
      row_pos[eq] = nd.base + j;
      row_cell[nd.base + j] = var_cell[eq];
    }
  }
  std::vector<int> Uf(F.Ubuf.size());
  for (size_t e = 0; e < F.Ubuf.size(); ++e) Uf[e] = row_pos[F.Ubuf[e]];
  LuDev& d = D.d;
  d.n = F.n;
  d.var_cell = B.upload(var_cell);
  d.row_cell = B.upload(row_cell);
  d.M = B.upload(F.Mbuf);
  d.V = B.upload(F.Vbuf);
  d.W = B.upload(F.Wbuf);
  // one trailing entry so that a node's list start is a valid index even when
  // it has no later variables (the sweeps load it unconditionally)
  std::vector<int> Upad(F.Ubuf);
  Upad.push_back(0);
  Uf.push_back(0);
  d.U = B.upload(Upad);
  d.Uf = B.upload(Uf);
  if (fp32) {
    d.M32 = B.upload(std::vector<float>(F.Mbuf.begin(), F.Mbuf.end()));
    d.V32 = B.upload(std::vector<float>(F.Vbuf.begin(), F.Vbuf.end()));
    d.W32 = B.upload(std::vector<float>(F.Wbuf.begin(), F.Wbuf.end()));
  }
  d.y = B.alloc<double>(F.n);
  d.z = B.alloc<double>(F.n);
  d.x = B.alloc<double>(F.n);
  D.height = F.max_height;
}

// Task lists of a factorization for a given number of factor entries per
// lane (epl): per-height lists of all nodes and the subtree grouping of the
// low heights.  Arrays go to B.
void make_schedule(const SupernodalLU& F, DevLU& D, double epl, DevBuf& B) {
  const int ns = (int)F.nodes.size();
  // g lanes per row: the largest power of two leaving more than epl entries per lane
  auto lanes_for = [epl](double len) {
    int g = 1;
    while (g < 64 && 2.0 * epl * g <= len) g <<= 1;
    return g;
  };
  auto log2i = [](int g) {
    int l = 0;
    while ((1 << l) < g) ++l;
    return l;
  };
  // Subtrees: the nodes below height hcut, grouped under the highest ancestor
  // below hcut, run in one launch (one workgroup per subtree).  hcut is the
  // highest cut that leaves at least kMinSub subtrees and at most kMaxRounds
  // sequential task rounds in any subtree.
  constexpr int kMinSub = 256, kMaxRounds = 24, kWaves = 8;
  auto single_tasks = [&](const SnNode& nd, bool fwd) {
    const int g = fwd ? lanes_for(nd.p) : lanes_for(0.5 * nd.p + nd.q);
    const int rows = fwd ? nd.p + nd.q : nd.p;
    return (rows + 64 / g - 1) / (64 / g);
  };
  int hcut = 0;
  std::vector<int> root_of(ns, -1);
  for (int hc = F.max_height; hc >= 2; --hc) {
    std::vector<int> rt(ns, -1);
    int nroots = 0;
    for (int s = ns - 1; s >= 0; --s) {  // parents come after children: walk from the top
      const SnNode& nd = F.nodes[s];
      if (nd.height >= hc) continue;
      const int par = nd.parent;
      if (par < 0 || F.nodes[par].height >= hc) {
        rt[s] = s;
        ++nroots;
      } else {
        rt[s] = rt[par];
      }
    }
    if (nroots < kMinSub) continue;
    std::map<int, std::vector<int>> per;  // root -> tasks per height
    for (int s = 0; s < ns; ++s)
      if (rt[s] >= 0) {
        auto& v = per[rt[s]];
        v.resize(hc, 0);
        v[F.nodes[s].height] += single_tasks(F.nodes[s], true);
      }
    int worst = 0;
    for (auto& kv : per) {
      int rounds = 0;
      for (int c : kv.second) rounds += (c + kWaves - 1) / kWaves;
      worst = std::max(worst, rounds);
    }
    if (worst <= kMaxRounds) {
      hcut = hc;
      root_of = rt;
      break;
    }
  }
  LuSub& SB = D.sub;
  SB.hcut = hcut;
  SB.nsub = 0;
  if (hcut >= 2) {
    std::vector<int> roots;
    for (int s = 0; s < ns; ++s)
      if (root_of[s] == s) roots.push_back(s);
    std::map<int, int> rindex;
    for (size_t i = 0; i < roots.size(); ++i) rindex[roots[i]] = (int)i;
    // members of each subtree by height
    std::vector<std::vector<std::vector<int>>> mem(roots.size(), std::vector<std::vector<int>>(hcut));
    for (int s = 0; s < ns; ++s)
      if (root_of[s] >= 0) mem[rindex[root_of[s]]][F.nodes[s].height].push_back(s);
    auto build = [&](bool multi, LuSubList& L) {
      std::vector<LuTask> ft, bt;
      std::vector<int2> fl, bl;
      std::vector<int> fp(1, 0), bp(1, 0);
      for (size_t i = 0; i < roots.size(); ++i) {
        for (int h = 0; h < hcut; ++h) {
          if (mem[i][h].empty()) continue;
          const int b0 = (int)ft.size();
          for (int s : mem[i][h]) {
            const SnNode& nd = F.nodes[s];
            if (multi) {
              for (int r = 0; r < nd.p + nd.q; r += kMrRows)
                ft.push_back(LuTask{nd.offM, nd.offV, nd.offU, nd.base, nd.p, nd.q, r, 0, 0});
            } else {
              const int g = lanes_for(nd.p), lg = log2i(g);
              for (int r = 0; r < nd.p + nd.q; r += 64 / g)
                ft.push_back(LuTask{nd.offM, nd.offV, nd.offU, nd.base, nd.p, nd.q, r, lg, 0});
            }
          }
          fl.push_back(make_int2(b0, (int)ft.size()));
        }
        fp.push_back((int)fl.size());
        for (int h = hcut - 1; h >= 0; --h) {
          if (mem[i][h].empty()) continue;
          const int b0 = (int)bt.size();
          for (int s : mem[i][h]) {
            const SnNode& nd = F.nodes[s];
            if (multi) {
              for (int r = 0; r < nd.p; r += kMrRows)
                bt.push_back(LuTask{nd.offM, nd.offW, nd.offU, nd.base, nd.p, nd.q, r, 0, 0});
            } else {
              const int g = lanes_for(0.5 * nd.p + nd.q), lg = log2i(g);
              for (int r = 0; r < nd.p; r += 64 / g)
                bt.push_back(LuTask{nd.offM, nd.offW, nd.offU, nd.base, nd.p, nd.q, r, lg, 0});
            }
          }
          bl.push_back(make_int2(b0, (int)bt.size()));
        }
        bp.push_back((int)bl.size());
      }
      L.ftask = B.upload(ft);
      L.flev = B.upload(fl);
      L.fptr = B.upload(fp);
      L.btask = B.upload(bt);
      L.blev = B.upload(bl);
      L.bptr = B.upload(bp);
    };
    build(false, SB.single);
    build(true, SB.multi);
    SB.nsub = (int)roots.size();
  }
  // entries per lane loaded per round: rows hold between epl and 2 epl entries
  // per lane (fewer when short, more only at 64 lanes per row); at most 8 to
  // bound the registers of the two pipeline stages
  const int kc = epl <= 2.0 ? 4 : 8;
  SB.kc = kc;
  D.tasks.assign(F.max_height + 1, LuTasks{});
  for (int h = 0; h <= F.max_height; ++h) {
    std::vector<LuTask> ft, bt, fm, bm;
    for (int s = 0; s < ns; ++s) {
      const SnNode& nd = F.nodes[s];
      if (nd.height != h) continue;
      const int gf = lanes_for(nd.p), lgf = log2i(gf);
      for (int r = 0; r < nd.p + nd.q; r += 64 / gf)
        ft.push_back(LuTask{nd.offM, nd.offV, nd.offU, nd.base, nd.p, nd.q, r, lgf, 0});
      const int gb = lanes_for(0.5 * nd.p + nd.q), lgb = log2i(gb);
      for (int r = 0; r < nd.p; r += 64 / gb)
        bt.push_back(LuTask{nd.offM, nd.offW, nd.offU, nd.base, nd.p, nd.q, r, lgb, 0});
      // multi-RHS: kMrRows consecutive rows of one node per wavefront
      for (int r = 0; r < nd.p + nd.q; r += kMrRows)
        fm.push_back(LuTask{nd.offM, nd.offV, nd.offU, nd.base, nd.p, nd.q, r, 0, 0});
      for (int r = 0; r < nd.p; r += kMrRows)
        bm.push_back(LuTask{nd.offM, nd.offW, nd.offU, nd.base, nd.p, nd.q, r, 0, 0});
    }
    LuTasks& T = D.tasks[h];
    T.kc = kc;
    T.nF = (int)ft.size();
    T.nB = (int)bt.size();
    T.ftask = B.upload(ft);
    T.btask = B.upload(bt);
    T.nFm = (int)fm.size();
    T.nBm = (int)bm.size();
    T.ftask_m = B.upload(fm);
    T.btask_m = B.upload(bm);
  }
}

// Tickets a wavefront of the one-launch sweeps takes at a time (one atomic on
// the shared ticket counter per batch).
constexpr int kFlowBatch = 4;

// The one-launch sweeps of a factorization (lu_flow.hpp): the same
// single-RHS tasks as make_schedule's, every height in ticket order (forward
// ascending, backward descending), with the node of each task, the tasks per
// node, and the nodes each waits on (forward: children; backward: the parent).
void make_flow(const SupernodalLU& F, DevLU& D, double epl, DevBuf& B) {
  const int ns = (int)F.nodes.size();
  auto lanes_for = [epl](double len) {
    int g = 1;
    while (g < 64 && 2.0 * epl * g <= len) g <<= 1;
    return g;
  };
  auto log2i = [](int g) {
    int l = 0;
    while ((1 << l) < g) ++l;
    return l;
  };
  const int kc = epl <= 2.0 ? 4 : 8;
  {
    std::vector<LuTask> ft, bt;
    std::vector<int> fn, bn, needf(ns, 0), needb(ns, 0);
    for (int h = 0; h <= F.max_height; ++h)
      for (int s = 0; s < ns; ++s) {
        const SnNode& nd = F.nodes[s];
        if (nd.height != h) continue;
        const int gf = lanes_for(nd.p), lgf = log2i(gf);
        for (int r = 0; r < nd.p + nd.q; r += 64 / gf) {
          ft.push_back(LuTask{nd.offM, nd.offV, nd.offU, nd.base, nd.p, nd.q, r, lgf, 0});
          fn.push_back(s);
          ++needf[s];
        }
      }
    for (int h = F.max_height; h >= 0; --h)
      for (int s = 0; s < ns; ++s) {
        const SnNode& nd = F.nodes[s];
        if (nd.height != h) continue;
        const int gb = lanes_for(0.5 * nd.p + nd.q), lgb = log2i(gb);
        for (int r = 0; r < nd.p; r += 64 / gb) {
          bt.push_back(LuTask{nd.offM, nd.offW, nd.offU, nd.base, nd.p, nd.q, r, lgb, 0});
          bn.push_back(s);
          ++needb[s];
        }
      }
    std::vector<std::vector<int>> kids(ns);
    for (int s = 0; s < ns; ++s) {
      const int par = F.nodes[s].parent;
      if (par >= 0) {
        if (F.nodes[par].height <= F.nodes[s].height) fail(CC_EDEVICE, "supernode tree: parent not above child");
        kids[par].push_back(s);
      }
    }
    std::vector<int> fptr(ns + 1, 0), fw, bptr(ns + 1, 0), bw;
    for (int s = 0; s < ns; ++s) {
      fptr[s + 1] = fptr[s] + (int)kids[s].size();
      for (int c : kids[s]) fw.push_back(c);
      const int par = F.nodes[s].parent;
      bptr[s + 1] = bptr[s] + (par >= 0 ? 1 : 0);
      if (par >= 0) bw.push_back(par);
    }
    LuFlow& W = D.flow;
    W.ncounters = 2 * ns + 2;
    W.counters = B.alloc<int>((size_t)W.ncounters);
    W.err = B.alloc<int>(1);
    HIPCHK(hipMemset(W.err, 0, sizeof(int)));
    W.ftask = B.upload(ft);
    W.btask = B.upload(bt);
    W.fwd.ntask = (int)ft.size();
    W.fwd.node = B.upload(fn);
    W.fwd.wait_ptr = B.upload(fptr);
    W.fwd.wait = fw.empty() ? B.alloc<int>(1) : B.upload(fw);
    W.fwd.need = B.upload(needf);
    W.fwd.done = W.counters;
    W.fwd.ticket = W.counters + 2 * ns;
    W.fwd.err = W.err;
    W.bwd.ntask = (int)bt.size();
    W.bwd.node = B.upload(bn);
    W.bwd.wait_ptr = B.upload(bptr);
    W.bwd.wait = bw.empty() ? B.alloc<int>(1) : B.upload(bw);
    W.bwd.need = B.upload(needb);
    W.bwd.done = W.counters + ns;
    W.bwd.ticket = W.counters + 2 * ns + 1;
    W.bwd.err = W.err;
    W.fwd.batch = W.bwd.batch = kFlowBatch;
    W.kc = kc;
    // waits give up after 50 ms of the device's wall clock (a sweep takes well
    // under a millisecond; the bound only ends a launch that cannot progress)
    int dev = 0, khz = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    W.limit = (long long)std::max(khz, 1) * 50;
  }
}


// Allocate a Work for nb right-hand sides (FP64 outer arrays, level arrays in
// T, factorization vectors in T on levels m < M and FP64 on the coarsest).
template <class T>
void alloc_work(cc_problem* P, Work<T>& W, int nb) {
  W.release();
  const int M = (int)P->dev.size() - 1;
  W.nb = nb;
  for (int m = 0; m <= M; ++m) {
    const long long n3 = cube(P->dev[m].st.n);
    W.s.push_back(W.own.template alloc<T>((size_t)n3 * nb));
    W.e.push_back(W.own.template alloc<T>((size_t)n3 * nb));
    W.et.push_back(W.own.template alloc<T>((size_t)n3 * nb));
    LuDev d = P->dev[m].lu.d;
    const size_t nv = (size_t)std::max(d.n, 1) * nb;
    d.y = d.z = d.x = nullptr;
    d.y32 = d.z32 = d.x32 = nullptr;
    if (std::is_same<T, float>::value && m < M) {
      d.y32 = W.own.template alloc<float>(nv);
      d.z32 = W.own.template alloc<float>(nv);
      d.x32 = W.own.template alloc<float>(nv);
    } else {
      d.y = W.own.template alloc<double>(nv);
      d.z = W.own.template alloc<double>(nv);
      d.x = W.own.template alloc<double>(nv);
    }
    W.lu.push_back(d);
  }
  W.s0 = W.own.template alloc<double>((size_t)cube(P->dev[0].st.n) * nb);
  W.norm = W.own.template alloc<unsigned long long>((size_t)nb);
}

void upload(cc_problem* P) {
  DevBuf& B = P->buf;
  const int M = (int)P->lv.size() - 1;

  P->dev.resize(P->lv.size());
  for (int m = 0; m <= M; ++m) {
    const LevelHost& L = *P->lv[m];
    DevLevel& D = P->dev[m];
    D.st.n = L.n;
    D.st.inv12h2 = 1.0 / (12.0 * L.h * L.h);
    for (int a = 0; a < 6; ++a) {
      D.st.bc[a] = L.wall_bc[a];
      for (int ly = 0; ly < 2; ++ly)
        for (int q = 0; q < 4; ++q) D.st.rob[a][ly][q] = L.wall[a].lay[ly][q];
    }
    D.st.type = B.upload(L.type);
    default_stencil_schedule(L.n, D.st.march, D.st.kz);
    // zone 1: phi_2 cells, and phi_1 cells with a phi_2 cell within 3 cells along
    // an axis (every cell a regular row reads, ghost fills included, lies there)
    D.st.zone = nullptr;
    D.near = nullptr;
    D.n_near = 0;
    if (!L.phi2.empty()) {
      const int nn = L.n;
      std::vector<uint8_t> zone((size_t)nn * nn * nn, 0);
      std::vector<int> near;
      for (int c : L.phi2) zone[c] = 1;
      for (int c : L.unknowns) {
        if (L.type[c] != kPhi1) continue;
        int ii[3];
        L.ijk(c, ii[0], ii[1], ii[2]);
        bool hit = false;
        for (int d = 0; d < 3 && !hit; ++d)
          for (int o = -3; o <= 3 && !hit; ++o) {
            if (o == 0) continue;
            int q[3] = {ii[0], ii[1], ii[2]};
            q[d] += o;
            if (q[d] < 0 || q[d] >= nn) continue;
            hit = L.type[L.idx(q[0], q[1], q[2])] == kPhi2;
          }
        if (hit) {
          zone[c] = 1;
          near.push_back(c);
        }
      }
      D.st.zone = B.upload(zone);
      D.near = B.upload(near);
      D.n_near = (int)near.size();
    }
    const int N2 = (int)L.phi2.size();
    std::vector<int> cols((size_t)N2 * kPLG);
    std::vector<double> vals((size_t)N2 * kPLG);
    std::vector<uint64_t> mask(N2, 0);
    for (int r = 0; r < N2; ++r)
      for (int t = 0; t < kPLG; ++t) {
        int c = L.plg_cols[(size_t)r * kPLG + t];
        cols[(size_t)t * N2 + r] = c;
        vals[(size_t)t * N2 + r] = L.plg_vals[(size_t)r * kPLG + t];
        if (L.type[c] == kPhi2) mask[r] |= (1ull << t);
      }
    D.plg.N2 = N2;
    D.plg.cell = B.upload(L.phi2);
    D.plg.cols = B.upload(cols);
    D.plg.vals = B.upload(vals);
    D.plg.vals32 = B.upload(std::vector<float>(vals.begin(), vals.end()));
    D.plg.phi2 = B.upload(mask);
    const SupernodalLU& F = P->lu[m];
    std::vector<int> orig = (m < M) ? L.phi2 : L.unknowns;
    std::vector<int> row_pos;
    upload_lu(P, F, orig, m < M, D.lu, row_pos);
    std::vector<int> nd(N2, 0);
    if (m < M)
      for (int r = 0; r < N2; ++r) nd[r] = row_pos[F.iperm[r]];
    D.plg.nd = B.upload(nd);
    size_t n3 = (size_t)L.n * L.n * L.n;
    D.s = B.alloc<double>(n3);
    D.e = B.alloc<double>(n3);
    D.et = B.alloc<double>(n3);
    std::vector<int2> ab;
    for (size_t c = 0; c < n3; ++c)
      if (L.host[c] >= 0 && L.host[c] != (int)c) ab.push_back(make_int2((int)c, L.host[c]));
    D.n_absorbed = (int)ab.size();
    D.absorbed = B.upload(ab);
  }
  P->d_norm = B.alloc<unsigned long long>(1);
  P->d_partial = B.alloc<double>(kReductionScratch);
  size_t n3 = (size_t)P->lv[0]->n * P->lv[0]->n * P->lv[0]->n;
  P->s0 = B.alloc<double>(n3);
  P->e0 = B.alloc<double>(n3);
  // FP64 single right-hand side: the level arrays themselves
  Work<double>& W = P->w64;
  W.nb = 1;
  for (int m = 0; m <= M; ++m) {
    W.s.push_back(P->dev[m].s);
    W.e.push_back(P->dev[m].e);
    W.et.push_back(P->dev[m].et);
    W.lu.push_back(P->dev[m].lu.d);
  }
  W.s0 = P->s0;
  W.norm = P->d_norm;
  // Sweep schedule per factorization (the autotuner): for 2 to 32 factor
  // entries per lane, each with and without the subtree launch and with at
  // most 2048, 4096, 8192 or any number of wavefronts per height launch, time
  // one LU solve on this device (the work vectors' contents do not matter) and
  // keep the fastest; the task lists of the other candidates are freed.
  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  for (int m = 0; m <= M; ++m) {
    DevLU& L = P->dev[m].lu;
    const long long n3m = cube(P->dev[m].st.n);
    float best = 1e30f;
    DevLU keep = L;
    DevBuf keep_buf;
    for (double epl : {2.0, 4.0, 8.0, 16.0, 32.0}) {
      DevBuf cand;
      make_schedule(P->lu[m], L, epl, cand);
      for (int on = 0; on < (L.sub.nsub > 0 ? 2 : 1); ++on)
        for (int wcap : {1 << 30, 8192, 4096, 2048}) {
          L.sub_on = on != 0;
          for (LuTasks& T : L.tasks) T.wcap = wcap;
          lu_sweeps<double, double>(P->stream, L, L.d, P->dev[m].et, n3m, 1);
          HIPCHK(hipEventRecord(ev0, P->stream));
          for (int rep = 0; rep < 5; ++rep) lu_sweeps<double, double>(P->stream, L, L.d, P->dev[m].et, n3m, 1);
          HIPCHK(hipEventRecord(ev1, P->stream));
          HIPCHK(hipGetLastError());
          HIPCHK(hipEventSynchronize(ev1));
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, ev0, ev1));
          {
            int k = 0;
            while (k < 4 && (2 << k) < (int)epl) ++k;
            float& slot = L.tune_ms[2 * k + on];
            slot = slot > 0.f ? std::min(slot, t / 5.0f) : t / 5.0f;
          }
          if (t < best) {
            best = t;
            keep = L;
            keep.epl = epl;
            keep.wcap = wcap;
          }
        }
      if (keep.epl == epl) {
        keep_buf.release();
        keep_buf = std::move(cand);
      } else {
        cand.release();
      }
    }
    std::copy(L.tune_ms, L.tune_ms + 10, keep.tune_ms);
    L = keep;
    P->dev[m].sched = std::move(keep_buf);
  }
  // Regular-row kernel schedule per level (the stencil autotuner): one cell per
  // thread, or the z-marching kernels with 4, 8, 16 or 32 planes per workgroup
  // in the linear or the XCD-aware tile order; 5 FP64 SMO-1 sweeps of each
  // timed on this device in 3 interleaved rounds after an untimed one, each
  // schedule's best round kept, the fastest schedule chosen (every schedule
  // gives the same result).  Interleaving and the best of rounds keep clock
  // ramps and cache warm-up from deciding between schedules a few percent apart.
  constexpr int kRounds = 3;
  for (int m = 0; m <= M; ++m) {
    DevLevel& D = P->dev[m];
    StencilLevel& S = D.st;
    const int kz0 = S.kz;
    float tmin[kStencilTrials];
    for (int c = 0; c < kStencilTrials; ++c) tmin[c] = 1e30f;
    for (int round = 0; round <= kRounds; ++round)
      for (int c = 0; c < kStencilTrials; ++c) {
        const int march = c == 0 ? 0 : (c <= 4 ? 1 : 2);
        const int kz = c == 0 ? kz0 : (2 << ((c - 1) % 4 + 1));      // 4, 8, 16, 32
        if (march && kz > S.n) continue;
        S.march = march;
        S.kz = kz;
        launch_smo1<double>(S, P->prm.omega, D.s, D.e, D.et, 1, P->stream);
        HIPCHK(hipEventRecord(ev0, P->stream));
        for (int rep = 0; rep < 5; ++rep) launch_smo1<double>(S, P->prm.omega, D.s, D.e, D.et, 1, P->stream);
        HIPCHK(hipEventRecord(ev1, P->stream));
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventSynchronize(ev1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, ev0, ev1));
        if (round > 0) tmin[c] = std::min(tmin[c], t);
      }
    float best = 1e30f;
    int bm = 0, bk = kz0;
    for (int c = 0; c < kStencilTrials; ++c) {
      const int march = c == 0 ? 0 : (c <= 4 ? 1 : 2);
      const int kz = c == 0 ? kz0 : (2 << ((c - 1) % 4 + 1));
      D.stencil_tune_us[c] = tmin[c] < 1e29f ? tmin[c] * 1000.f / 5.f : 0.f;
      if (tmin[c] < best) {
        best = tmin[c];
        bm = march;
        bk = kz;
      }
    }
    // the grid-size default (linear order, the plane count that gives ~4096
    // workgroups) unless another schedule's best round is 3% faster: bursts of
    // 5 sweeps rank schedules a few percent apart differently from the solve's
    // launches (at 256^3, 8 and 16 planes within 1-3% in the trials, 131
    // against 122 us in 50 back-to-back launches)
    int dm, dk;
    default_stencil_schedule(S.n, dm, dk);
    const int cd = dm == 0 ? 0 : 1 + (dk == 4 ? 0 : dk == 8 ? 1 : dk == 16 ? 2 : 3);
    if ((dm == 0 || dk == 4 || dk == 8 || dk == 16 || dk == 32) && tmin[cd] < 1e29f && best > 0.97f * tmin[cd]) {
      bm = dm;
      bk = dm == 0 ? kz0 : dk;
    }
    S.march = D.tuned_march = bm;
    S.kz = D.tuned_kz = bk;
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
}

// ---------------------------------------------------------------- solve steps
template <class T>
T* vec_y(const LuDev& F);
template <>
double* vec_y<double>(const LuDev& F) { return F.y; }
template <>
float* vec_y<float>(const LuDev& F) { return F.y32; }

// SMO-2 on level m < M: b_2 = s_2 - L21 e_1, e_2 = L22^-1 b_2 (Sec. 5.3)
template <class T>
void smo2(cc_problem* P, const Work<T>& W, int m, const T* s, T* e, int nb) {
  DevLevel& D = P->dev[m];
  if (D.plg.N2 == 0) return;
  const LuDev& F = W.lu[m];
  const long long n3 = cube(D.st.n);
  launch_plg_b2<T>(D.plg, s, e, vec_y<T>(F), n3, nb, P->stream);
  lu_sweeps<T, T>(P->stream, D.lu, F, e, n3, nb);
}

// e = L^(M)^-1 s on the coarsest level, in FP64 whatever T is
template <class T>
void bottom(cc_problem* P, const Work<T>& W, const T* s, T* e, int nb) {
  const int M = (int)P->dev.size() - 1;
  DevLevel& D = P->dev[M];
  const LuDev& F = W.lu[M];
  const long long n3 = cube(D.st.n);
  launch_zero<T>(e, n3 * nb, P->stream);
  launch_gather<T, double>(F.n, F.row_cell, s, n3, F.y, nb, P->stream);
  lu_sweeps<double, T>(P->stream, D.lu, F, e, n3, nb);
}

// e = VCycle(s) on level m (e overwritten); tmp is a work array of the level.
template <class T>
void vcycle(cc_problem* P, const Work<T>& W, int m, const T* s, T* e, T* tmp, int nb) {
  const int M = (int)P->dev.size() - 1;
  if (m == M) {
    bottom<T>(P, W, s, e, nb);
    return;
  }
  DevLevel& D = P->dev[m];
  const long long n3 = cube(D.st.n);
  const double om = P->prm.omega;
  T* cur = e;
  T* oth = tmp;
  // SMO-1 after an SMO-2 splits in two: the far sweep (rows that read no phi_2
  // cell) needs only the previous SMO-1, so it runs on the side stream beside
  // the LU-correction; the near sweep follows the LU-correction on the main
  // stream, and the next SMO-2 waits for both.
  const bool split = P->overlap && D.st.zone && P->stream2;
  auto smoothing = [&](int nu) {
    for (int it = 0; it < nu; ++it) {
      const bool more = it + 1 < nu;
      if (more && split) {
        HIPCHK(hipEventRecord(P->ev_fork, P->stream));
        HIPCHK(hipStreamWaitEvent(P->stream2, P->ev_fork, 0));
        launch_smo1_far<T>(D.st, om, s, cur, oth, nb, P->stream2);
        HIPCHK(hipEventRecord(P->ev_join, P->stream2));
      }
      smo2<T>(P, W, m, s, cur, nb);
      if (!more) break;
      if (split) {
        launch_smo1_near<T>(D.st, om, s, cur, oth, D.near, D.n_near, nb, P->stream);
        HIPCHK(hipStreamWaitEvent(P->stream, P->ev_join, 0));
      } else {
        launch_smo1<T>(D.st, om, s, cur, oth, nb, P->stream);
      }
      std::swap(cur, oth);
    }
  };
  if (P->prm.nu1 == 0) {
    launch_zero<T>(e, n3 * nb, P->stream);
  } else {
    // from e = 0 the first sweep is e = omega D^-1 s (no stencil reads)
    launch_smo1_first<T>(D.st, om, s, oth, nb, P->stream);
    std::swap(cur, oth);
    smoothing(P->prm.nu1);
  }
  DevLevel& C = P->dev[m + 1];
  launch_restrict<T>(D.st, C.st, s, cur, W.s[m + 1], nb, P->stream);
  vcycle<T>(P, W, m + 1, W.s[m + 1], W.e[m + 1], W.et[m + 1], nb);
  // merged coarse cells take their host's value before the prolongation
  launch_copy_pairs<T>(C.n_absorbed, C.absorbed, W.e[m + 1], cube(C.st.n), nb, P->stream);
  launch_prolong_add<T>(D.st, C.st.n, W.e[m + 1], cur, nb, P->stream);
  if (P->prm.nu2 > 0) {
    launch_smo1<T>(D.st, om, s, cur, oth, nb, P->stream);
    std::swap(cur, oth);
    smoothing(P->prm.nu2);
  }
  if (cur != e) HIPCHK(hipMemcpyAsync(e, cur, n3 * nb * sizeof(T), hipMemcpyDeviceToDevice, P->stream));
}

// s = r - L x on level m for nb arrays (FP64)
void residual(cc_problem* P, int m, const double* r, const double* x, double* s, int nb = 1) {
  DevLevel& D = P->dev[m];
  launch_stencil_residual(D.st, r, x, s, nb, P->stream);
  launch_plg_residual(D.plg, r, x, s, 0, nb, cube(D.st.n), P->stream);
}

// Full multigrid (Sec. 5, algorithm FMG) in FP64, its recursion unrolled: each
// level's right-hand side is coarse_rhs[m - 1] (the same problem assembled on
// that level) or, with coarse_rhs null, the restriction of the finer one; the
// coarsest level is solved by its LU, and from the coarsest level up each
// level's solution is the interpolated coarser one improved by `cycles`
// V-cycles (level residual, V-cycle correction, update).  phi receives the
// level-0 result; merged cells take their host's value.  nb right-hand sides
// at a stride of n_m^3 (W sized for nb); the coarse right-hand sides of the
// group start coarse_off arrays into coarse_rhs[m - 1].
// crhs[m], cx[m] (m = 1..M, nb * n_m^3 doubles each): the coarse levels'
// right-hand side (used only without coarse_rhs) and solution arrays; every
// cell of each is written before it is read.  With start in [1, M), the
// ascent begins at level `start` from the iterate cx[start] holds (improved
// by `cycles` V-cycles there) instead of the coarsest level's LU solution.
void fmg(cc_problem* P, const Work<double>& W, const double* r, const double* const* coarse_rhs, long long coarse_off,
         double* phi, int cycles, int nb, const std::vector<double*>& crhs, const std::vector<double*>& cx,
         int start = -1) {
  const int M = (int)P->dev.size() - 1;
  const int s0 = (start >= 1 && start < M) ? start : M;
  std::vector<const double*> rhs(M + 1);
  std::vector<double*> x(M + 1);
  rhs[0] = r;
  x[0] = phi;
  for (int m = 1; m <= M; ++m) {
    rhs[m] = coarse_rhs ? coarse_rhs[m - 1] + coarse_off * cube(P->dev[m].st.n) : crhs[m];
    x[m] = cx[m];
  }
  if (!coarse_rhs)
    for (int m = 0; m < s0; ++m)
      launch_fmg_restrict(P->dev[m].st, P->dev[m + 1].st, rhs[m], crhs[m + 1], nb, P->stream);
  if (s0 == M) {
    bottom<double>(P, W, rhs[M], x[M], nb);
  } else {
    for (int c = 0; c < cycles; ++c) {
      residual(P, s0, rhs[s0], x[s0], W.s[s0], nb);
      vcycle<double>(P, W, s0, W.s[s0], W.e[s0], W.et[s0], nb);
      launch_add_unknowns<double>(P->dev[s0].st, W.e[s0], nullptr, x[s0], nb, P->stream);
    }
  }
  for (int m = s0 - 1; m >= 0; --m) {
    DevLevel& D = P->dev[m];
    launch_fmg_prolong(D.st, P->dev[m + 1].st, x[m + 1], x[m], nb, P->stream);
    for (int c = 0; c < cycles; ++c) {
      residual(P, m, rhs[m], x[m], W.s[m], nb);
      vcycle<double>(P, W, m, W.s[m], W.e[m], W.et[m], nb);
      launch_add_unknowns<double>(D.st, W.e[m], nullptr, x[m], nb, P->stream);
    }
  }
  launch_copy_pairs<double>(P->dev[0].n_absorbed, P->dev[0].absorbed, phi, cube(P->dev[0].st.n), nb, P->stream);
}

// The coarse arrays of cc_fmg / cc_fmg_batched: allocated by the handle at the
// first call (and grown for a larger group), kept until cc_destroy.
void fmg_alloc(cc_problem* P, int nb) {
  const int M = (int)P->dev.size() - 1;
  if ((int)P->fmg_rhs.size() == M + 1 && P->fmg_nb >= nb) return;
  for (int m = 1; m < (int)P->fmg_rhs.size(); ++m) {
    P->buf.free(P->fmg_rhs[m]);
    P->buf.free(P->fmg_x[m]);
  }
  P->fmg_rhs.assign(M + 1, nullptr);
  P->fmg_x.assign(M + 1, nullptr);
  for (int m = 1; m <= M; ++m) {
    P->fmg_rhs[m] = P->buf.alloc<double>((size_t)cube(P->dev[m].st.n) * nb);
    P->fmg_x[m] = P->buf.alloc<double>((size_t)cube(P->dev[m].st.n) * nb);
  }
  P->fmg_nb = nb;
}

std::vector<double> read_norms(cc_problem* P, const unsigned long long* d, int nb) {
  std::vector<unsigned long long> bits(nb);
  HIPCHK(hipMemcpyAsync(bits.data(), d, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, P->stream));
  HIPSYNC(P->stream);
  std::vector<double> v(nb);
  for (int b = 0; b < nb; ++b) std::memcpy(&v[b], &bits[b], sizeof(double));
  return v;
}
double read_norm(cc_problem* P) { return read_norms(P, P->d_norm, 1)[0]; }

// One outer iteration after the residual s0 and its norms are current:
// FP64: phi += VCycle(s0).  Mixed (defect correction): d = s0 / |s0| in FP32,
// phi += |s0| VCycle32(d).  Then s0 = r - L phi and its norms.
template <class T>
void outer_step(cc_problem* P, const Work<T>& W, const double* r, double* phi, int nb) {
  DevLevel& D0 = P->dev[0];
  const long long n3 = cube(D0.st.n);
  if constexpr (std::is_same<T, double>::value) {
    vcycle<T>(P, W, 0, W.s0, W.e[0], W.et[0], nb);
    launch_add_unknowns<T>(D0.st, W.e[0], nullptr, phi, nb, P->stream);
  } else {
    launch_scale_residual<T>(n3, W.s0, W.norm, W.s[0], nb, P->stream);
    vcycle<T>(P, W, 0, W.s[0], W.e[0], W.et[0], nb);
    launch_add_unknowns<T>(D0.st, W.e[0], W.norm, phi, nb, P->stream);
  }
  residual(P, 0, r, phi, W.s0, nb);
  launch_zero_u64(W.norm, nb, P->stream);
  launch_maxabs(W.s0, n3, nb, W.norm, P->d_partial, P->stream);
}

struct SolveRec {
  int iterations = 0;
  double rel = 0.0;
  std::vector<double> hist;
};

// The prologue of the multigrid iteration (Sec. 5.3) on nb right-hand sides:
// the right-hand side norms rn (a zero one sets its phi to 0), phi masked to
// the unknowns, the residual and its norms sn; records started.  Returns
// whether every member has converged already.
bool update_rec(cc_problem* P, const std::vector<double>& rn, const std::vector<double>& sn, std::vector<SolveRec>& rec,
                bool first) {
  bool all = true;
  for (size_t b = 0; b < rn.size(); ++b) {
    double rel = rn[b] > 0 ? sn[b] / rn[b] : 0.0;
    rec[b].rel = rel;
    rec[b].hist.push_back(rel);
    if (!first) ++rec[b].iterations;
    if (!(rel < P->prm.tol)) all = false;
    if (!std::isfinite(rel)) fail(CC_ENOCONV, "non-finite residual");
  }
  return all;
}

template <class T>
bool loop_prologue(cc_problem* P, Work<T>& W, const double* r, double* phi, int nb, std::vector<double>& rn,
                   std::vector<SolveRec>& rec) {
  DevLevel& D0 = P->dev[0];
  const long long n3 = cube(D0.st.n);
  launch_zero_u64(W.norm, nb, P->stream);
  launch_maxabs(r, n3, nb, W.norm, P->d_partial, P->stream);
  rn = read_norms(P, W.norm, nb);
  for (int b = 0; b < nb; ++b) {
    if (!std::isfinite(rn[b])) fail(CC_EINVAL, "non-finite right-hand side");
    // L is nonsingular: r = 0 has the solution 0, whatever the guess (the relative
    // stopping test is undefined there)
    if (rn[b] == 0.0) launch_zero<double>(phi + (long long)b * n3, n3, P->stream);
  }
  launch_mask_unknowns(D0.st, phi, nb, P->stream);
  residual(P, 0, r, phi, W.s0, nb);
  launch_zero_u64(W.norm, nb, P->stream);
  launch_maxabs(W.s0, n3, nb, W.norm, P->d_partial, P->stream);
  std::vector<double> sn = read_norms(P, W.norm, nb);
  rec.assign(nb, SolveRec{});
  return update_rec(P, rn, sn, rec, true);
}

// The captured outer step for (r, phi, nb), kept across solves with the same arrays.
template <class T>
void ensure_graph(cc_problem* P, Work<T>& W, const double* r, double* phi, int nb) {
  if (W.g_r == r && W.g_phi == phi && W.g_nb == nb && W.gexec) return;
  W.drop_graph();
  HIPCHK(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
  outer_step<T>(P, W, r, phi, nb);
  HIPCHK(hipStreamEndCapture(P->stream, &W.graph));
  HIPCHK(hipGraphInstantiate(&W.gexec, W.graph, nullptr, nullptr, 0));
  W.g_r = r;
  W.g_phi = phi;
  W.g_nb = nb;
}

// The multigrid iteration of Sec. 5.3 on nb right-hand sides at once (r, phi:
// nb * n^3, batch-major) until every relative residual is below tol or max_iter.
template <class T>
void solve_loop(cc_problem* P, Work<T>& W, const double* r, double* phi, int nb, std::vector<SolveRec>& rec) {
  DevLevel& D0 = P->dev[0];
  const long long n3 = cube(D0.st.n);
  std::vector<double> rn;
  bool done = loop_prologue<T>(P, W, r, phi, nb, rn, rec);
  const bool use_graph = P->prm.use_graph != 0;
  if (use_graph && !done) ensure_graph<T>(P, W, r, phi, nb);
  int it = 0;
  while (!done && it < P->prm.max_iter) {
    if (use_graph)
      HIPCHK(hipGraphLaunch(W.gexec, P->stream));
    else
      outer_step<T>(P, W, r, phi, nb);
    std::vector<double> sn = read_norms(P, W.norm, nb);
    ++it;
    done = update_rec(P, rn, sn, rec, false);
  }
  launch_copy_pairs<double>(D0.n_absorbed, D0.absorbed, phi, n3, nb, P->stream);
  HIPSYNC(P->stream);
}

// Restarted flexible GMRES(k), right-preconditioned by one V-cycle per
// iteration (cc_params.krylov = k > 0; FP64, or the FP32 V-cycle on the
// max-norm-scaled vector in mixed precision): an acceleration of the multigrid
// iteration, also for geometries where the plain iteration does not contract.
// The Krylov vectors, the outer residual, the max-norm test and the iteration
// count (V-cycles) are FP64 as in the plain iteration.
void gmres_loop(cc_problem* P, const double* r, double* phi, SolveRec& rec) {
  Work<double>& W = P->w64;
  DevLevel& D0 = P->dev[0];
  const long long n3 = cube(D0.st.n);
  const int k = P->prm.krylov;
  const bool mixed = P->prm.precision == CC_MIXED;
  if (mixed && P->w32.nb < 1) alloc_work(P, P->w32, 1);
  Krylov& K = P->kr;
  if (K.k != k) {
    K.own.release();
    K.k = k;
    K.V = K.own.alloc<double>((size_t)(k + 1) * n3);
    K.Z = K.own.alloc<double>((size_t)k * n3);
    K.w = K.own.alloc<double>((size_t)n3);
    K.d = K.own.alloc<double>((size_t)k + 2);
    K.amax = K.own.alloc<unsigned long long>(1);
  }
  hipStream_t st = P->stream;
  auto norm2 = [&](const double* w) {  // (w, w)
    launch_dots_norm(n3, w, w, n3, 0, K.d, P->d_partial, st);
    double q = 0.0;
    HIPCHK(hipMemcpyAsync(&q, K.d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPSYNC(st);
    return q;
  };
  auto put = [&](const std::vector<double>& c) {
    HIPCHK(hipMemcpyAsync(K.d, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPSYNC(st);
  };
  auto maxabs = [&](const double* v) {
    launch_zero_u64(P->d_norm, 1, st);
    launch_maxabs(v, n3, 1, P->d_norm, P->d_partial, st);
    return read_norm(P);
  };
  const double rn = maxabs(r);
  if (!std::isfinite(rn)) fail(CC_EINVAL, "non-finite right-hand side");
  if (rn == 0.0) launch_zero<double>(phi, n3, st);  // r = 0: the solution is 0
  launch_mask_unknowns(D0.st, phi, 1, st);
  const double nunk = (double)P->lv[0]->unknowns.size();
  rec = SolveRec{};
  int cycles = 0;
  for (;;) {
    residual(P, 0, r, phi, W.s0, 1);
    const double rel = rn > 0 ? maxabs(W.s0) / rn : 0.0;
    rec.hist.push_back(rel);
    rec.rel = rel;
    if (!std::isfinite(rel)) fail(CC_ENOCONV, "non-finite residual");
    if (rel < P->prm.tol || cycles >= P->prm.max_iter) break;
    const double beta = std::sqrt(norm2(W.s0));
    put({1.0 / beta});
    launch_combo(n3, W.s0, n3, 1, K.d, K.V, 0, nullptr, nullptr, P->d_partial, st);
    std::vector<std::vector<double>> Hb(k + 1, std::vector<double>(k, 0.0));  // unrotated
    std::vector<std::vector<double>> R(k + 1, std::vector<double>(k, 0.0));   // rotated
    std::vector<double> cs(k), sn(k), g(k + 1, 0.0);
    g[0] = beta;
    int j = 0;
    bool converged = false;
    auto solve_y = [&](int m) {
      std::vector<double> y(m, 0.0);
      for (int i = m - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < m; ++l) t -= R[i][l] * y[l];
        y[i] = t / R[i][i];
      }
      return y;
    };
    while (j < k && cycles < P->prm.max_iter) {
      double* vj = K.V + (long long)j * n3;
      double* zj = K.Z + (long long)j * n3;
      if (mixed) {
        // z = max|v| * VCycle32(v / max|v|): the FP32 V-cycle as preconditioner
        Work<float>& W32 = P->w32;
        launch_zero_u64(P->d_norm, 1, st);
        launch_maxabs(vj, n3, 1, P->d_norm, P->d_partial, st);
        launch_scale_residual<float>(n3, vj, P->d_norm, W32.s[0], 1, st);
        vcycle<float>(P, W32, 0, W32.s[0], W32.e[0], W32.et[0], 1);
        launch_zero<double>(zj, n3, st);
        launch_add_unknowns<float>(D0.st, W32.e[0], P->d_norm, zj, 1, st);
      } else {
        vcycle<double>(P, W, 0, vj, zj, W.et[0], 1);
      }
      ++cycles;
      launch_stencil_apply(D0.st, zj, K.w, st);
      launch_plg_residual(D0.plg, nullptr, zj, K.w, 1, 1, n3, st);
      // classical Gram-Schmidt (projections and |w| in one pass, the update and
      // the new |w| in another); a second pass only when the norm drops by more
      // than 1/sqrt(2) (Daniel-Gragg-Kaufman-Stewart criterion)
      auto project = [&](std::vector<double>& h) {  // returns |w|^2 before
        launch_dots_norm(n3, K.w, K.V, n3, j + 1, K.d, P->d_partial, st);
        std::vector<double> hw(j + 2);
        HIPCHK(hipMemcpyAsync(hw.data(), K.d, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPSYNC(st);
        h.assign(hw.begin(), hw.begin() + j + 1);
        return hw[j + 1];
      };
      auto subtract = [&](const std::vector<double>& h) {  // w -= V h; returns |w|^2 after
        put(h);
        launch_combo(n3, K.V, n3, j + 1, K.d, K.w, 2, nullptr, K.d + k + 1, P->d_partial, st);
        double q = 0.0;
        HIPCHK(hipMemcpyAsync(&q, K.d + k + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPSYNC(st);
        return q;
      };
      std::vector<double> h, h2;
      const double wn0 = std::sqrt(project(h));
      double hn = std::sqrt(subtract(h));
      if (hn < 0.7071 * wn0) {
        project(h2);
        hn = std::sqrt(subtract(h2));
        for (int i = 0; i <= j; ++i) h[i] += h2[i];
      }
      for (int i = 0; i <= j; ++i) Hb[i][j] = R[i][j] = h[i];
      Hb[j + 1][j] = R[j + 1][j] = hn;
      if (hn > 0) {
        put({1.0 / hn});
        launch_combo(n3, K.w, n3, 1, K.d, K.V + (long long)(j + 1) * n3, 0, nullptr, nullptr, P->d_partial, st);
      }
      for (int i = 0; i < j; ++i) {
        const double a = R[i][j], b = R[i + 1][j];
        R[i][j] = cs[i] * a + sn[i] * b;
        R[i + 1][j] = -sn[i] * a + cs[i] * b;
      }
      const double a = R[j][j], b = R[j + 1][j], den = std::hypot(a, b);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? b / den : 0.0;
      R[j][j] = den;
      R[j + 1][j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++j;
      const double est = std::fabs(g[j]);
      // |res|_inf >= |res|_2 / sqrt(N): the max-norm test can pass only if
      if (est <= P->prm.tol * rn * std::sqrt(nunk) || hn == 0.0) {
        // residual vector V_{j+1} (beta e1 - Hb y), its max-norm
        std::vector<double> y = solve_y(j), c(j + 1, 0.0);
        c[0] = beta;
        for (int i = 0; i <= j; ++i)
          for (int l = 0; l < j; ++l) c[i] -= Hb[i][l] * y[l];
        put(c);
        launch_zero_u64(K.amax, 1, st);
        launch_combo(n3, K.V, n3, j + 1, K.d, nullptr, 0, K.amax, nullptr, P->d_partial, st);
        unsigned long long bits = 0;
        HIPCHK(hipMemcpyAsync(&bits, K.amax, sizeof(bits), hipMemcpyDeviceToHost, st));
        HIPSYNC(st);
        double res;
        std::memcpy(&res, &bits, sizeof(res));
        if (res < P->prm.tol * rn || hn == 0.0) {
          converged = true;
          break;
        }
      }
    }
    std::vector<double> y = solve_y(j);
    put(y);
    launch_combo(n3, K.Z, n3, j, K.d, phi, 1, nullptr, nullptr, P->d_partial, st);
    (void)converged;
  }
  rec.iterations = cycles;
  launch_copy_pairs<double>(D0.n_absorbed, D0.absorbed, phi, n3, 1, st);
  HIPSYNC(st);
}

void fill_info(const SolveRec& rc, double seconds, cc_solve_info* info) {
  if (!info) return;
  info->iterations = rc.iterations;
  info->rel_residual = rc.rel;
  info->history_len = (int)std::min<size_t>(rc.hist.size(), CC_HISTORY_MAX);
  for (int i = 0; i < info->history_len; ++i) info->history[i] = rc.hist[i];
  info->seconds = seconds;
}

FieldDesc to_desc(const cc_field* f) {
  FieldDesc d;
  if (!f) return d;
  d.kind = f->kind;
  d.n_terms = f->n_terms;
  int per = 0;
  switch (f->kind) {
    case CC_FIELD_ZERO: per = 0; break;
    case CC_FIELD_POLY: per = 4 * f->n_terms; break;
    case CC_FIELD_SINPROD: per = 7; break;
    case CC_FIELD_EXPCOS: per = 5; break;
    case CC_FIELD_GAUSS: per = 5 * f->n_terms; break;
    case CC_FIELD_XSINEXP: per = 1; break;
    default: fail(CC_EINVAL, "unknown field kind");
  }
  if (per > kFieldMax || per < 0) fail(CC_EINVAL, "field has too many terms");
  if (per > 0 && !f->data) fail(CC_EINVAL, "field data is NULL");
  for (int i = 0; i < per; ++i) d.d[i] = f->data[i];
  if (f->kind == CC_FIELD_POLY)
    for (int t = 0; t < f->n_terms; ++t) {
      int a = (int)d.d[4 * t], b = (int)d.d[4 * t + 1], c = (int)d.d[4 * t + 2];
      if (a < 0 || b < 0 || c < 0 || a + b + c > 4) fail(CC_EINVAL, "polynomial field of degree > 4");
    }
  return d;
}

// average of a field (value, or d/dn = side * d/dx_axis) over a wall face square
double face_average(const LevelHost& L, const FieldDesc& g, int cell, int axis, int side, bool normal_deriv) {
  static thread_local std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(8, gx, gw);
  int ii[3];
  L.ijk(cell, ii[0], ii[1], ii[2]);
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = L.origin[a] + L.h * ii[a];
    hi[a] = lo[a] + L.h;
  }
  double xw = L.origin[axis] + (side > 0 ? L.n * L.h : 0.0);
  int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
  double acc = 0.0;
  for (int p = 0; p < 8; ++p)
    for (int q = 0; q < 8; ++q) {
      double x[3];
      x[axis] = xw;
      x[a1] = 0.5 * (lo[a1] + hi[a1]) + 0.5 * L.h * gx[p];
      x[a2] = 0.5 * (lo[a2] + hi[a2]) + 0.5 * L.h * gx[q];
      double v;
      if (normal_deriv) {
        double gr[3];
        field_grad(g, x[0], x[1], x[2], gr);
        v = side * gr[axis];
      } else {
        v = field_value(g, x[0], x[1], x[2], 0);
      }
      acc += gw[p] * gw[q] * v;
    }
  return 0.25 * acc;
}

// The datum of the wall face of `cell` on wall (axis, side): Dirichlet <g>,
// Neumann <dg/dn>, Robin <alpha g + beta dg/dn> (n out of the box).
double wall_datum(const LevelHost& L, const FieldDesc& g, int cell, int axis, int side) {
  const int w = 2 * axis + (side > 0 ? 1 : 0);
  const int bc = L.wall_bc[w];
  if (bc == CC_DIRICHLET) return face_average(L, g, cell, axis, side, false);
  if (bc == CC_NEUMANN) return face_average(L, g, cell, axis, side, true);
  const double* ab = L.dom->wall_robin[w];
  return ab[0] * face_average(L, g, cell, axis, side, false) + ab[1] * face_average(L, g, cell, axis, side, true);
}

}  // namespace
}  // namespace cc

using namespace cc;

template <class F>
static int guard(F&& f) {
  try {
    f();
    return CC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return CC_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CC_EINVAL;
  }
}

extern "C" {

const char* cc_last_error(void) { return g_last_error.c_str(); }

void cc_default_params(cc_params* p) {
  if (!p) return;
  p->theta = 0.1;
  p->omega = 0.8;
  p->nu1 = 3;
  p->nu2 = 3;
  p->n_min = 16;
  p->max_iter = 200;
  p->tol = 1e-10;
  p->precision = CC_FP64;
  p->leaf_size = 64;
  p->device = 0;
  p->use_graph = 1;
  p->krylov = 0;
  p->pivot_tol = 1e-14;
  p->fit_on_device = 1;
}

int cc_build(const cc_domain* dom, const cc_params* prm, void* stream, cc_problem** out) {
  return guard([&] {
    if (!dom || !prm || !out) fail(CC_EINVAL, "null argument");
    *out = nullptr;
    if (dom->n < 8) fail(CC_EINVAL, "n must be at least 8");
    // cell indices are 32-bit (host arrays, FV-PLG column lists): n^3 < 2^31
    if (dom->n > 1290) fail(CC_EINVAL, "n must be at most 1290 (32-bit cell indices)");
    if (std::fabs(dom->h * dom->n - 1.0) > 1e-12) fail(CC_EINVAL, "h must equal 1/n");
    if (dom->n_obst < 0 || (dom->n_obst > 0 && !dom->obst)) fail(CC_EINVAL, "bad obstacle list");
    if (!(prm->theta > 0 && prm->theta < 0.5)) fail(CC_EINVAL, "theta must lie in (0, 1/2)");
    if (!(prm->omega > 0 && prm->omega < 2)) fail(CC_EINVAL, "omega must lie in (0, 2)");
    if (prm->nu1 < 0 || prm->nu2 < 0 || prm->max_iter < 0 || prm->n_min < 8 || prm->leaf_size < 1)
      fail(CC_EINVAL, "bad multigrid parameters");
    if (prm->precision != CC_FP64 && prm->precision != CC_MIXED) fail(CC_EINVAL, "precision must be CC_FP64 or CC_MIXED");
    if (prm->krylov < 0 || prm->krylov > 64) fail(CC_EINVAL, "krylov must lie in [0, 64]");
    if (!(prm->pivot_tol > 0 && prm->pivot_tol <= 1e6)) fail(CC_EINVAL, "pivot_tol must lie in (0, 1e6]");
    if (prm->fit_on_device != 0 && prm->fit_on_device != 1) fail(CC_EINVAL, "fit_on_device must be 0 or 1");
    for (int a = 0; a < 6; ++a) {
      if (dom->wall_bc[a] != CC_DIRICHLET && dom->wall_bc[a] != CC_NEUMANN && dom->wall_bc[a] != CC_ROBIN)
        fail(CC_EINVAL, "bad wall bc");
      if (dom->wall_bc[a] == CC_ROBIN) {
        const double al = dom->wall_robin[a][0], be = dom->wall_robin[a][1];
        if (!(std::isfinite(al) && std::isfinite(be)) || (al == 0.0 && be == 0.0))
          fail(CC_EINVAL, "a Robin wall needs finite (alpha, beta), not both 0");
      }
    }
    auto P = std::make_unique<cc_problem>();
    P->prm = *prm;
    P->device = prm->device;
    DomainSpec& D = P->dom;
    D.n = dom->n;
    D.h = dom->h;
    for (int a = 0; a < 3; ++a) D.origin[a] = dom->origin[a];
    for (int a = 0; a < 6; ++a) {
      D.wall_bc[a] = dom->wall_bc[a];
      D.wall_robin[a][0] = dom->wall_bc[a] == CC_ROBIN ? dom->wall_robin[a][0] : 0.0;
      D.wall_robin[a][1] = dom->wall_bc[a] == CC_ROBIN ? dom->wall_robin[a][1] : 0.0;
    }
    for (int t = 0; t < dom->n_obst; ++t) {
      const cc_obstacle& o = dom->obst[t];
      Obstacle ob;
      if (o.kind != CC_ELLIPSOID && o.kind != CC_TORUS) fail(CC_EINVAL, "obstacle kind must be CC_ELLIPSOID or CC_TORUS");
      ob.kind = o.kind;
      for (int a = 0; a < 3; ++a) {
        ob.c[a] = o.center[a];
        ob.axes[a] = o.axes[a];
        if (o.kind == CC_ELLIPSOID && !(o.axes[a] > 0)) fail(CC_EINVAL, "semi-axes must be positive");
      }
      if (o.kind == CC_TORUS) {
        ob.radii[0] = o.radii[0];
        ob.radii[1] = o.radii[1];
        if (!(std::isfinite(o.radii[0]) && o.radii[1] > 0 && o.radii[0] > o.radii[1]))
          fail(CC_EINVAL, "a torus needs radii R > r > 0");
      }
      for (int a = 0; a < 9; ++a) ob.rot[a] = o.rot[a];
      for (int a = 0; a < 3; ++a)
        if (!std::isfinite(ob.c[a])) fail(CC_EINVAL, "obstacle centre must be finite");
      // rot's columns are the semi-axis directions: orthonormal (the bounding
      // sphere of radius max(axes) holds only for a rotation)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double d = 0.0;
          for (int i = 0; i < 3; ++i) d += ob.rot[3 * i + a] * ob.rot[3 * i + b];
          if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-9)) fail(CC_EINVAL, "obstacle rot must be orthonormal");
        }
      if (o.bc != CC_DIRICHLET && o.bc != CC_NEUMANN && o.bc != CC_ROBIN) fail(CC_EINVAL, "bad obstacle bc");
      ob.bc = o.bc;
      if (o.bc == CC_ROBIN) {
        ob.alpha = o.robin[0];
        ob.beta = o.robin[1];
        if (!(std::isfinite(ob.alpha) && std::isfinite(ob.beta)) || (ob.alpha == 0.0 && ob.beta == 0.0))
          fail(CC_EINVAL, "a Robin condition needs finite (alpha, beta), not both 0");
      }
      if (o.kind == CC_TORUS) {
        ob.R = ob.radii[0] + ob.radii[1];
        ob.ls.poly = true;
        ob.ls.p = torus_poly(ob.c, ob.radii[0], ob.radii[1], ob.rot);
      } else {
        ob.R = std::max(ob.axes[0], std::max(ob.axes[1], ob.axes[2]));
        ob.ls.q = ellipsoid_quadric(ob.c, ob.axes, ob.rot);
      }
      D.obst.push_back(ob);
    }
    if (dom->inside != 0 && dom->inside != 1) fail(CC_EINVAL, "inside must be 0 or 1");
    D.inside = dom->inside == 1;
    if (D.inside) {
      // Omega = the obstacle's interior: negate its quadric so that Omega = {q > 0}
      if (D.obst.size() != 1) fail(CC_EINVAL, "an interior domain is bounded by exactly one obstacle");
      if (D.obst[0].kind != CC_ELLIPSOID) fail(CC_EINVAL, "an interior domain is bounded by an ellipsoid");
      Quadric& q = D.obst[0].ls.q;
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) q.Q[i][j] = -q.Q[i][j];
        q.b[i] = -q.b[i];
      }
      q.c = -q.c;
    }
    std::vector<int> sizes = {D.n};
    while (sizes.back() % 2 == 0 && sizes.back() / 2 >= prm->n_min) sizes.push_back(sizes.back() / 2);
    const int M = (int)sizes.size() - 1;
    P->lv.resize(sizes.size());
    P->lu.resize(sizes.size());
    P->lu_mat.resize(sizes.size());
    P->setup_s.resize(sizes.size());
    P->lu_s.resize(sizes.size());
    if (P->device >= 0) {
      HIPCHK(hipSetDevice(P->device));
      {  // resolve this device's copy of the allocation-free entry points' scratch
        double* s = nullptr;
        long long c = 0;
        noalloc_scratch(P->device, &s, &c);
      }
      if (stream) {
        P->stream = (hipStream_t)stream;
      } else {
        HIPCHK(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
        P->own_stream = true;
      }
      // the side stream of the far SMO-1 sweeps (default priority) and its events
      HIPCHK(hipStreamCreateWithFlags(&P->stream2, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
    }
    // the FV-PLG least-squares fits on the device (a handle with a device and
    // fit_on_device), else on the host
    struct DeviceLsq : PlgLsqSolver {
      hipStream_t st;
      void solve(int nsys, const int* off, const double* A, const double* ell, double* y, int* ok) override {
        plg_lsq_device(nsys, off, A, ell, y, ok, st);
      }
    } dlsq;
    dlsq.st = P->stream;
    PlgLsqSolver* lsq = (P->device >= 0 && prm->fit_on_device) ? &dlsq : nullptr;
    try {
      for (int m = 0; m <= M; ++m) {
        double t0 = now_s();
        P->lv[m] = std::make_unique<LevelHost>();
        P->lv[m]->build(D, sizes[m], prm->theta, lsq);
        const double t1 = now_s();
        std::vector<std::array<int, 3>> xyz;
        std::vector<int> orig;
        build_lu_matrix(*P->lv[m], m == M, P->lu_mat[m], xyz, orig);
        factorize(P->lu_mat[m], xyz, prm->leaf_size, prm->pivot_tol, P->lu[m]);
        P->setup_s[m] = now_s() - t0;
        P->lu_s[m] = now_s() - t1;
      }
      if (P->device >= 0) upload(P.get());
    } catch (...) {
      P->buf.release();
      if (P->own_stream) (void)hipStreamDestroy(P->stream);
      if (P->stream2) (void)hipStreamDestroy(P->stream2);
      if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
      if (P->ev_join) (void)hipEventDestroy(P->ev_join);
      throw;
    }
    *out = P.release();
  });
}

int cc_num_levels(const cc_problem* p) { return p ? (int)p->lv.size() : 0; }

int cc_get_level_info(const cc_problem* p, int level, cc_level_info* info) {
  return guard([&] {
    check_level(p, level);
    if (!info) fail(CC_EINVAL, "null info");
    const LevelHost& L = *p->lv[level];
    info->n = L.n;
    info->n_unknowns = (long long)L.unknowns.size();
    info->n_phi2 = (long long)L.phi2.size();
    info->n_cut = (long long)L.cut.size();
    info->n_merged = L.n_merged;
    info->lu_vars = p->lu[level].n;
    info->lu_entries = p->lu[level].entries();
    info->lu_nodes = (int)p->lu[level].nodes.size();
    info->lu_depth = p->lu[level].max_height + 1;
    info->setup_seconds = p->setup_s[level];
    info->lu_seconds = p->lu_s[level];
    const bool dev = p->device >= 0 && (int)p->dev.size() > level;
    const bool on = dev && p->dev[level].lu.sub_on;
    info->lu_subtree_cut = on ? p->dev[level].lu.sub.hcut : 0;
    info->lu_subtrees = on ? p->dev[level].lu.sub.nsub : 0;
    info->lu_entries_per_lane = dev ? (int)p->dev[level].lu.epl : 0;
    info->lu_waves_cap = dev && p->dev[level].lu.wcap < (1 << 30) ? p->dev[level].lu.wcap : 0;
    for (int k = 0; k < 10; ++k) info->lu_tune_ms[k] = dev ? p->dev[level].lu.tune_ms[k] : 0.0;
    info->n_near = dev ? p->dev[level].n_near : 0;
    info->stencil_march = dev ? p->dev[level].st.march : 0;
    info->stencil_planes = dev ? p->dev[level].st.kz : 0;
    for (int k = 0; k < kStencilTrials; ++k) info->stencil_tune_us[k] = dev ? p->dev[level].stencil_tune_us[k] : 0.0;
  });
}

int cc_export_cells(const cc_problem* p, int level, unsigned char* type, int* host, double* volfrac) {
  return guard([&] {
    check_level(p, level);
    const LevelHost& L = *p->lv[level];
    size_t n3 = L.type.size();
    double h3 = L.h * L.h * L.h;
    for (size_t c = 0; c < n3; ++c) {
      if (type) type[c] = L.type[c];
      if (host) host[c] = L.host[c];
      if (volfrac) volfrac[c] = L.vol[c] / h3;
    }
  });
}

int cc_fit_patches(const cc_problem* p, int level, const cc_field* u, int* cell, int* axis, double* coef,
                   double* exact, double* fitted) {
  return guard([&] {
    check_level(p, level);
    FieldDesc fd = to_desc(u);
    fit_cut_cells(*p->lv[level], p->dom, fd, cell, axis, coef, exact, fitted);
  });
}

int cc_export_plg(const cc_problem* p, int level, int* row_cell, int* cols, double* vals) {
  return guard([&] {
    check_level(p, level);
    const LevelHost& L = *p->lv[level];
    if (row_cell) std::copy(L.phi2.begin(), L.phi2.end(), row_cell);
    if (cols) std::copy(L.plg_cols.begin(), L.plg_cols.end(), cols);
    if (vals) std::copy(L.plg_vals.begin(), L.plg_vals.end(), vals);
  });
}

int cc_selfcheck_lu(const cc_problem* p, int level, double* rel_residual) {
  return guard([&] {
    check_level(p, level);
    if (!rel_residual) fail(CC_EINVAL, "null output");
    *rel_residual = p->lu[level].n ? selfcheck(p->lu_mat[level], p->lu[level], 12345u) : 0.0;
  });
}

int cc_export_lu_nodes(const cc_problem* p, int level, int* base, int* np, int* nq, int* height, int* parent) {
  return guard([&] {
    check_level(p, level);
    const SupernodalLU& F = p->lu[level];
    for (size_t s = 0; s < F.nodes.size(); ++s) {
      const SnNode& nd = F.nodes[s];
      if (base) base[s] = nd.base;
      if (np) np[s] = nd.p;
      if (nq) nq[s] = nd.q;
      if (height) height[s] = nd.height;
      if (parent) parent[s] = nd.parent;
    }
  });
}

// r = f - N g on level `level` for nf fields at once (Sec. 2.4): cell averages of
// f_k (or of Delta f_k) on the device; the cut-cell integrals of f_k on the
// device too, from each cut cell's quadrature rule built on the host as line
// pieces (one rule serves every field); on the host, the patch data of g_k
// (when any g_k is nonzero), the merged groups' averages, the wall-ghost terms
// of regular rows and the boundary sites of FV-PLG rows; the host results
// reach the device as sparse overwrites (special and absorbed cells) and
// additions (boundary terms), so no full array crosses PCIe.  r_dev holds nf
// arrays of n_m^3 at stride n_m^3.
static void assemble_rhs(cc_problem* p, int level, int nf, const std::vector<FieldDesc>& fds, int f_mode,
                         const std::vector<FieldDesc>& gds, double* r_dev) {
  const LevelHost& L = *p->lv[level];
  const int n = L.n;
  const double h = L.h;
  const long long n3 = (long long)n * n * n;
  for (int k = 0; k < nf; ++k) launch_cell_average(n, h, L.origin, fds[k], f_mode, 8, r_dev + k * n3, p->stream);
  const double s12 = 1.0 / (12.0 * h * h);
  const double h3 = h * h * h;
  // full cells inside merged groups: their device averages
  std::vector<int> special;
  for (int c : L.unknowns)
    if (L.cut.count(c) || L.groups.count(c)) special.push_back(c);
  std::vector<int> full_members;
  {
    std::vector<int> tmp;
    for (int c : special)
      for (int m : L.members(c, tmp))
        if (!L.cut.count(m)) full_members.push_back(m);
    std::sort(full_members.begin(), full_members.end());
    full_members.erase(std::unique(full_members.begin(), full_members.end()), full_members.end());
  }
  TempBuf tmpb;
  std::vector<double> fm_val((size_t)full_members.size() * nf);
  if (!full_members.empty()) {
    int* d_cells = tmpb.upload(full_members);
    double* d_vals = tmpb.alloc<double>(fm_val.size());
    launch_gather<double, double>((int)full_members.size(), d_cells, r_dev, n3, d_vals, nf, p->stream);
    HIPCHK(hipMemcpyAsync(fm_val.data(), d_vals, fm_val.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  }
  HIPSYNC(p->stream);
  std::map<int, size_t> fm_pos;
  for (size_t t = 0; t < full_members.size(); ++t) fm_pos[full_members[t]] = t;
  // per cut cell and field: the integral of f over the cut region (device) and
  // the patch datum of g (Dirichlet: <<g>>, Neumann: h <<dg/dn>>, Robin:
  // scaled; host), from one quadrature pass per cut cell, in chunks of cells
  std::vector<int> cuts;
  for (const auto& kv : L.cut) cuts.push_back(kv.first);
  std::vector<double> cut_int(cuts.size() * nf), cut_dat(cuts.size() * nf, 0.0);
  bool any_g = false;
  for (const FieldDesc& g : gds) any_g = any_g || g.kind != CC_FIELD_ZERO;
  static_assert(sizeof(LinePiece) == sizeof(PieceRec), "line piece layouts differ");
  if (!cuts.empty()) {
    const FieldDesc* d_f = tmpb.upload(fds);
    double* d_int = tmpb.alloc<double>(cut_int.size());
    const size_t kChunk = 8192;
    std::vector<std::vector<LinePiece>> pcs(std::min(kChunk, cuts.size()));
    for (size_t c0 = 0; c0 < cuts.size(); c0 += kChunk) {
      const size_t c1 = std::min(cuts.size(), c0 + kChunk);
#pragma omp parallel for schedule(dynamic, 8)
      for (long t = (long)c0; t < (long)c1; ++t) {
        int m = cuts[t];
        const CutData& cd = L.cut.at(m);
        const Obstacle& ob = p->dom.obst[cd.obst];
        int bc = ob.bc;
        int ii[3];
        L.ijk(m, ii[0], ii[1], ii[2]);
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = L.origin[a] + h * ii[a];
          hi[a] = lo[a] + h;
        }
        std::vector<LinePiece>& pc = pcs[t - c0];
        pc.clear();
        SurfaceSet sn;
        region_pieces(lo, hi, ob.ls, kQuadOrder, pc, any_g ? &sn : nullptr);
        if (!any_g) continue;
        // the datum in the scale of the site row: Neumann h <<dg/dn>>, Robin
        // h <<alpha g + beta dg/dn>> / (|alpha| h + |beta|)
        const double scale = bc == CC_NEUMANN ? h
                             : bc == CC_ROBIN  ? h / (std::fabs(ob.alpha) * h + std::fabs(ob.beta))
                                               : 1.0;
        for (int k = 0; k < nf; ++k) {
          double acc = 0.0, area = 0.0;
          for (size_t q = 0; q < sn.w.size(); ++q) {
            const double* x = &sn.x[3 * q];
            double v;
            if (bc == CC_DIRICHLET) {
              v = field_value(gds[k], x[0], x[1], x[2], 0);
            } else {
              double gr[3];
              field_grad(gds[k], x[0], x[1], x[2], gr);
              v = gr[0] * sn.n[3 * q] + gr[1] * sn.n[3 * q + 1] + gr[2] * sn.n[3 * q + 2];
              if (bc == CC_ROBIN) v = ob.alpha * field_value(gds[k], x[0], x[1], x[2], 0) + ob.beta * v;
            }
            acc += sn.w[q] * v;
            area += sn.w[q];
          }
          cut_dat[t * nf + k] = (area > 0) ? acc / area * scale : 0.0;
        }
      }
      std::vector<int> off(c1 - c0 + 1, 0);
      for (size_t t = c0; t < c1; ++t) {
        const size_t np = pcs[t - c0].size();
        if (off[t - c0] + np > (size_t)INT32_MAX) fail(CC_ENOMEM, "too many quadrature pieces in one chunk");
        off[t - c0 + 1] = off[t - c0] + (int)np;
      }
      std::vector<PieceRec> flat((size_t)off.back());
      for (size_t t = c0; t < c1; ++t)
        if (!pcs[t - c0].empty())
          std::memcpy(&flat[off[t - c0]], pcs[t - c0].data(), pcs[t - c0].size() * sizeof(PieceRec));
      TempBuf cb;
      const int* d_off = cb.upload(off);
      const PieceRec* d_pc = cb.upload(flat);
      launch_piece_integrals((int)(c1 - c0), d_off, d_pc, kQuadOrder, d_f, nf, f_mode, d_int + c0 * nf, p->stream);
      HIPSYNC(p->stream);
    }
    HIPCHK(hipMemcpy(cut_int.data(), d_int, cut_int.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  std::map<int, size_t> cut_pos;
  for (size_t t = 0; t < cuts.size(); ++t) cut_pos[cuts[t]] = t;
  auto cell_integral = [&](int m, int k) -> double {
    auto it = cut_pos.find(m);
    return (it == cut_pos.end()) ? fm_val[fm_pos.at(m) * nf + k] * h3 : cut_int[it->second * nf + k];
  };
  // overwrites: special cells (region averages), absorbed cells (0)
  std::vector<int> set_cells = special;
  std::vector<double> set_vals(special.size() * nf);
#pragma omp parallel for schedule(dynamic, 8)
  for (long t = 0; t < (long)special.size(); ++t) {
    int c = special[t];
    std::vector<int> tmp;
    const std::vector<int>& mem = L.members(c, tmp);
    double vol = 0.0;
    for (int m : mem) vol += L.vol[m];
    for (int k = 0; k < nf; ++k) {
      double tot = 0.0;
      for (int m : mem) tot += cell_integral(m, k);
      set_vals[t * nf + k] = tot / vol;
    }
  }
  for (long long c = 0; c < n3; ++c)
    if (L.host[c] != (int)c) {
      set_cells.push_back((int)c);
      for (int k = 0; k < nf; ++k) set_vals.push_back(0.0);
    }
  // additions: wall-ghost terms of regular rows, boundary sites of FV-PLG rows
  std::vector<int> wall_cells;
  for (int c : L.unknowns) {
    if (L.type[c] != kPhi1) continue;
    int ii[3];
    L.ijk(c, ii[0], ii[1], ii[2]);
    bool near = false;
    for (int d = 0; d < 3; ++d) near = near || ii[d] <= 1 || ii[d] >= n - 2;
    if (near) wall_cells.push_back(c);
  }
  const int N2 = (int)L.phi2.size();
  std::vector<int> add_cells = wall_cells;
  add_cells.insert(add_cells.end(), L.phi2.begin(), L.phi2.end());
  std::vector<double> add_vals(add_cells.size() * nf, 0.0);
#pragma omp parallel for schedule(dynamic, 64)
  for (long t = 0; t < (long)wall_cells.size(); ++t) {
    int c = wall_cells[t];
    int ii[3];
    L.ijk(c, ii[0], ii[1], ii[2]);
    for (int k = 0; k < nf; ++k) {
      double corr = 0.0;
      for (int d = 0; d < 3; ++d)
        for (int side : {-1, 1}) {
          int layer = side > 0 ? n - 1 - ii[d] : ii[d];
          if (layer > 1) continue;
          const int w = 2 * d + (side > 0 ? 1 : 0);
          corr += L.wall[w].dat[layer] * s12 * wall_datum(L, gds[k], c, d, side);
        }
      add_vals[t * nf + k] = -corr;
    }
  }
  std::vector<std::vector<size_t>> by_row(N2);
  for (size_t s = 0; s < L.sites.size(); ++s) by_row[L.sites[s].row].push_back(s);
  const size_t w0 = wall_cells.size();
#pragma omp parallel for schedule(dynamic, 8)
  for (long rr = 0; rr < N2; ++rr) {
    for (int k = 0; k < nf; ++k) {
      double corr = 0.0;
      for (size_t si : by_row[rr]) {
        const Site& st = L.sites[si];
        double dat;
        if (st.kind == 'W') {
          dat = wall_datum(L, gds[k], st.cell, st.axis, st.side);
          if (st.bc == CC_NEUMANN) {
            dat *= h;
          } else if (st.bc == CC_ROBIN) {
            const double* ab = L.dom->wall_robin[2 * st.axis + (st.side > 0 ? 1 : 0)];
            dat *= h / (std::fabs(ab[0]) * h + std::fabs(ab[1]));
          }
        } else {
          dat = cut_dat[cut_pos.at(st.cell) * nf + k];
        }
        corr += st.coef * dat;
      }
      add_vals[(w0 + rr) * nf + k] = -corr;
    }
  }
  if (!set_cells.empty()) {
    int* d_c = tmpb.upload(set_cells);
    double* d_v = tmpb.upload(set_vals);
    launch_scatter_values((int)set_cells.size(), d_c, d_v, r_dev, n3, nf, 0, p->stream);
  }
  if (!add_cells.empty()) {
    int* d_c = tmpb.upload(add_cells);
    double* d_v = tmpb.upload(add_vals);
    launch_scatter_values((int)add_cells.size(), d_c, d_v, r_dev, n3, nf, 1, p->stream);
  }
  HIPSYNC(p->stream);
}

int cc_assemble_rhs_level(cc_problem* p, int level, const cc_field* f, int f_mode, const cc_field* g,
                          double* r_dev) {
  return guard([&] {
    if (!p || !r_dev) fail(CC_EINVAL, "null argument");
    check_level(p, level);
    need_device(p);
    if (f_mode != CC_VALUE && f_mode != CC_LAPLACIAN) fail(CC_EINVAL, "bad f_mode");
    HIPCHK(hipSetDevice(p->device));
    assemble_rhs(p, level, 1, {to_desc(f)}, f_mode, {to_desc(g)}, r_dev);
  });
}

int cc_assemble_rhs_batched(cc_problem* p, int level, int nf, const cc_field* f, int f_mode, const cc_field* g,
                            int g_per_field, double* r_dev) {
  return guard([&] {
    if (!p || !r_dev || !f || nf < 1) fail(CC_EINVAL, "bad argument");
    check_level(p, level);
    need_device(p);
    if (f_mode != CC_VALUE && f_mode != CC_LAPLACIAN) fail(CC_EINVAL, "bad f_mode");
    if (g_per_field != 0 && g_per_field != 1) fail(CC_EINVAL, "g_per_field must be 0 or 1");
    HIPCHK(hipSetDevice(p->device));
    std::vector<FieldDesc> fds(nf), gds(nf);
    for (int k = 0; k < nf; ++k) {
      fds[k] = to_desc(f + k);
      gds[k] = to_desc(g ? (g_per_field ? g + k : g) : nullptr);
    }
    assemble_rhs(p, level, nf, fds, f_mode, gds, r_dev);
  });
}

int cc_assemble_rhs(cc_problem* p, const cc_field* f, int f_mode, const cc_field* g, double* r_dev) {
  return cc_assemble_rhs_level(p, 0, f, f_mode, g, r_dev);
}

int cc_apply(cc_problem* p, int level, const double* x, double* y) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (!x || !y) fail(CC_EINVAL, "null array");
    DevLevel& D = p->dev[level];
    launch_stencil_apply(D.st, x, y, p->stream);
    launch_plg_residual(D.plg, nullptr, x, y, 1, 1, cube(D.st.n), p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_residual(cc_problem* p, int level, const double* r, const double* x, double* s, double* maxabs) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (!r || !x || !s) fail(CC_EINVAL, "null array");
    DevLevel& D = p->dev[level];
    residual(p, level, r, x, s);
    launch_zero_u64(p->d_norm, 1, p->stream);
    launch_maxabs(s, cube(D.st.n), 1, p->d_norm, p->d_partial, p->stream);
    double v = read_norm(p);
    if (maxabs) *maxabs = v;
  });
}

int cc_smo1(cc_problem* p, int level, const double* s, double* e) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (!s || !e) fail(CC_EINVAL, "null array");
    DevLevel& D = p->dev[level];
    long long n3 = (long long)D.st.n * D.st.n * D.st.n;
    launch_smo1<double>(D.st, p->prm.omega, s, e, D.et, 1, p->stream);
    HIPCHK(hipMemcpyAsync(e, D.et, n3 * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIPSYNC(p->stream);
  });
}

// A wait of a one-launch LU sweep that gave up (the launch then finished with
// wrong values) is reported by the next call that checks, and cleared.
static void flow_check(cc_problem* p) {
  for (size_t m = 0; m < p->dev.size(); ++m) {
    const DevLU& L = p->dev[m].lu;
    if (!L.flow_on || !L.flow.err) continue;
    int e = 0;
    HIPCHK(hipMemcpy(&e, L.flow.err, sizeof(int), hipMemcpyDeviceToHost));
    if (e) {
      HIPCHK(hipMemset(L.flow.err, 0, sizeof(int)));
      fail(CC_EDEVICE, "a wait of the one-launch LU sweep gave up on level " + std::to_string(m));
    }
  }
}

int cc_smo2(cc_problem* p, int level, const double* s, double* e) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (!s || !e) fail(CC_EINVAL, "null array");
    if (level == (int)p->lv.size() - 1) fail(CC_EINVAL, "the coarsest level has no LU-correction");
    smo2<double>(p, p->w64, level, s, e, 1);
    HIPSYNC(p->stream);
    flow_check(p);
  });
}

int cc_restrict(cc_problem* p, int level, const double* s, const double* e, double* sc) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (level + 1 >= (int)p->lv.size()) fail(CC_EINVAL, "no coarser level");
    if (!s || !e || !sc) fail(CC_EINVAL, "null array");
    launch_restrict<double>(p->dev[level].st, p->dev[level + 1].st, s, e, sc, 1, p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_prolong_add(cc_problem* p, int level, const double* ec, double* ef) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (level + 1 >= (int)p->lv.size()) fail(CC_EINVAL, "no coarser level");
    if (!ec || !ef) fail(CC_EINVAL, "null array");
    launch_prolong_add<double>(p->dev[level].st, p->dev[level + 1].st.n, ec, ef, 1, p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_fmg(cc_problem* p, const double* r, const double* const* coarse_rhs, double* phi, int cycles) {
  return guard([&] {
    if (!p || !r || !phi) fail(CC_EINVAL, "null argument");
    need_device(p);
    if (cycles < 1 || cycles > 64) fail(CC_EINVAL, "cycles must lie in [1, 64]");
    if (coarse_rhs)
      for (size_t m = 1; m < p->dev.size(); ++m)
        if (!coarse_rhs[m - 1]) fail(CC_EINVAL, "null coarse right-hand side");
    fmg_alloc(p, 1);
    fmg(p, p->w64, r, coarse_rhs, 0, phi, cycles, 1, p->fmg_rhs, p->fmg_x);
    HIPSYNC(p->stream);
    flow_check(p);
  });
}

int cc_fmg_noalloc(cc_problem* p, const double* r, const double* const* coarse_rhs, double* phi, int cycles) {
  return guard([&] {
    if (!p || !r || !phi) fail(CC_EINVAL, "null argument");
    need_device(p);
    if (cycles < 1 || cycles > 64) fail(CC_EINVAL, "cycles must lie in [1, 64]");
    if (coarse_rhs)
      for (size_t m = 1; m < p->dev.size(); ++m)
        if (!coarse_rhs[m - 1]) fail(CC_EINVAL, "null coarse right-hand side");
    HIPCHK(hipSetDevice(p->device));
    double* base = nullptr;
    long long cap = 0;
    noalloc_scratch(p->device, &base, &cap);
    // layout: the solution arrays of levels 1..M, then (without coarse_rhs) their
    // right-hand sides
    const int M = (int)p->dev.size() - 1;
    long long need = 0;
    for (int m = 1; m <= M; ++m) need += cube(p->dev[m].st.n);
    if (!coarse_rhs) need *= 2;
    if (need > cap)
      fail(CC_EINVAL, "cc_fmg_noalloc: the coarse levels need " + std::to_string(need) +
                          " doubles of scratch, more than the " + std::to_string(cap) + " it holds");
    std::vector<double*> cx(M + 1, nullptr), crhs(M + 1, nullptr);
    double* q = base;
    for (int m = 1; m <= M; ++m) {
      cx[m] = q;
      q += cube(p->dev[m].st.n);
    }
    if (!coarse_rhs)
      for (int m = 1; m <= M; ++m) {
        crhs[m] = q;
        q += cube(p->dev[m].st.n);
      }
    fmg(p, p->w64, r, coarse_rhs, 0, phi, cycles, 1, crhs, cx);
    HIPSYNC(p->stream);
  });
}

int cc_fmg_batched(cc_problem* p, int nrhs, const double* r, const double* const* coarse_rhs, double* phi,
                   int cycles) {
  return guard([&] {
    if (!p || !r || !phi || nrhs < 1) fail(CC_EINVAL, "bad argument");
    need_device(p);
    if (cycles < 1 || cycles > 64) fail(CC_EINVAL, "cycles must lie in [1, 64]");
    if (coarse_rhs)
      for (size_t m = 1; m < p->dev.size(); ++m)
        if (!coarse_rhs[m - 1]) fail(CC_EINVAL, "null coarse right-hand side");
    const int cap = std::min(nrhs, CC_BATCH_MAX);
    if (p->wb64.nb < cap) alloc_work(p, p->wb64, cap);
    fmg_alloc(p, cap);
    const long long n3 = cube(p->dev[0].st.n);
    for (int b0 = 0; b0 < nrhs; b0 += CC_BATCH_MAX) {
      const int nb = std::min(CC_BATCH_MAX, nrhs - b0);
      fmg(p, p->wb64, r + b0 * n3, coarse_rhs, b0, phi + b0 * n3, cycles, nb, p->fmg_rhs, p->fmg_x);
    }
    HIPSYNC(p->stream);
  });
}

int cc_fmg_restrict(cc_problem* p, int level, const double* s, double* sc) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (level + 1 >= (int)p->lv.size()) fail(CC_EINVAL, "no coarser level");
    if (!s || !sc) fail(CC_EINVAL, "null array");
    launch_fmg_restrict(p->dev[level].st, p->dev[level + 1].st, s, sc, 1, p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_fmg_prolong(cc_problem* p, int level, const double* xc, double* xf) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (level + 1 >= (int)p->lv.size()) fail(CC_EINVAL, "no coarser level");
    if (!xc || !xf) fail(CC_EINVAL, "null array");
    launch_fmg_prolong(p->dev[level].st, p->dev[level + 1].st, xc, xf, 1, p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_bottom_solve(cc_problem* p, const double* s, double* e) {
  return guard([&] {
    if (!p || !s || !e) fail(CC_EINVAL, "null argument");
    need_device(p);
    bottom<double>(p, p->w64, s, e, 1);
    HIPSYNC(p->stream);
    flow_check(p);
  });
}

int cc_vcycle(cc_problem* p, int level, const double* s, double* e) {
  return guard([&] {
    check_level(p, level);
    need_device(p);
    if (!s || !e) fail(CC_EINVAL, "null array");
    vcycle<double>(p, p->w64, level, s, e, p->dev[level].et, 1);
    HIPSYNC(p->stream);
    flow_check(p);
  });
}

int cc_solve(cc_problem* p, const double* r, double* phi, cc_solve_info* info) {
  int conv = 0;
  int rc = guard([&] {
    if (!p || !r || !phi) fail(CC_EINVAL, "null argument");
    need_device(p);
    double t0 = now_s();
    std::vector<SolveRec> rec;
    if (p->prm.krylov > 0) {
      rec.resize(1);
      gmres_loop(p, r, phi, rec[0]);
    } else if (p->prm.precision == CC_MIXED) {
      if (p->w32.nb < 1) alloc_work(p, p->w32, 1);
      solve_loop<float>(p, p->w32, r, phi, 1, rec);
    } else {
      solve_loop<double>(p, p->w64, r, phi, 1, rec);
    }
    flow_check(p);
    fill_info(rec[0], now_s() - t0, info);
    conv = (rec[0].rel < p->prm.tol) ? 1 : 0;
  });
  if (rc == CC_OK && !conv) {
    set_last_error("max_iter reached before tol");
    return CC_ENOCONV;
  }
  return rc;
}

// volume fractions of a level's cells on the device (uploaded on first use)
static void level_volfrac(cc_problem* p, int level) {
  if ((int)p->volfrac.size() <= level) p->volfrac.resize(level + 1, nullptr);
  if (p->volfrac[level]) return;
  const LevelHost& Lm = *p->lv[level];
  const long long m3 = cube(Lm.n);
  std::vector<float> vf(m3);
  const double h3 = Lm.h * Lm.h * Lm.h;
  for (long long c = 0; c < m3; ++c) vf[c] = (float)(Lm.vol[c] / h3);
  p->volfrac[level] = p->buf.upload(vf);
}

int cc_net_pairs(cc_problem* p, int level, int nrhs, const double* r, const double* phi, double phi_scale, float* x,
                 float* t, unsigned char* mask) {
  return guard([&] {
    if (!p || !r || !phi || !x || !t || !mask || nrhs < 1) fail(CC_EINVAL, "bad argument");
    need_device(p);
    check_level(p, level);
    if (!(phi_scale > 0)) fail(CC_EINVAL, "phi_scale must be positive");
    HIPCHK(hipSetDevice(p->device));
    const int m = p->lv[level]->n, n0 = p->lv[0]->n;
    level_volfrac(p, level);
    const long long n3 = cube(n0);
    for (int b0 = 0; b0 < nrhs; b0 += CC_BATCH_MAX) {
      const int nb = std::min(CC_BATCH_MAX, nrhs - b0);
      if (!p->pair_norm) p->pair_norm = p->buf.alloc<unsigned long long>(CC_BATCH_MAX);
      launch_zero_u64(p->pair_norm, nb, p->stream);
      launch_maxabs(r + b0 * n3, n3, nb, p->pair_norm, p->d_partial, p->stream);
      const long long o = (long long)b0 * cube(m);
      launch_net_pairs(n0, m, nb, r + b0 * n3, phi + b0 * n3, p->dev[0].st.type, p->pair_norm, p->volfrac[level],
                       phi_scale, x + 2 * o, t + o, mask + o, p->stream);
    }
    HIPSYNC(p->stream);
  });
}

int cc_learned_guess(cc_problem* p, cc_net* net, int level, double phi_scale, const double* r, double* phi) {
  return guard([&] {
    if (!p || !net || !r || !phi) fail(CC_EINVAL, "null argument");
    need_device(p);
    check_level(p, level);
    if (!(phi_scale > 0)) fail(CC_EINVAL, "phi_scale must be positive");
    const LevelHost& Lm = *p->lv[level];
    const int m = Lm.n, n0 = p->lv[0]->n;
    const long long m3 = cube(m);
    level_volfrac(p, level);
    if (p->net_cells < m3) {
      p->net_x = p->buf.alloc<float>(2 * m3);
      p->net_y = p->buf.alloc<float>(m3);
      p->net_cells = m3;
    }
    launch_zero_u64(p->d_norm, 1, p->stream);
    launch_maxabs(r, cube(n0), 1, p->d_norm, p->d_partial, p->stream);
    const double rn = read_norm(p);
    const double inv = rn > 0 ? 1.0 / rn : 0.0;
    launch_net_features(n0, m, r, inv, p->volfrac[level], p->net_x, p->stream);
    HIPSYNC(p->stream);
    int rc = cc_net_forward(net, m, 1, p->net_x, p->net_y);
    if (rc != CC_OK) fail(rc, cc_last_error());
    launch_prolong_trilinear(p->dev[0].st, m, p->net_y, rn / phi_scale, phi, p->stream);
    HIPSYNC(p->stream);
  });
}

int cc_learned_fmg(cc_problem* p, cc_net* net, int level, double phi_scale, const double* r,
                   const double* const* coarse_rhs, double* phi, int cycles) {
  return guard([&] {
    if (!p || !net || !r || !phi) fail(CC_EINVAL, "null argument");
    need_device(p);
    check_level(p, level);
    const int M = (int)p->lv.size() - 1;
    if (level < 1 || level >= M) fail(CC_EINVAL, "level must lie in [1, levels - 1)");
    if (!(phi_scale > 0)) fail(CC_EINVAL, "phi_scale must be positive");
    if (cycles < 1 || cycles > 16) fail(CC_EINVAL, "cycles must lie in [1, 16]");
    if (coarse_rhs)
      for (int m = 1; m <= M; ++m)
        if (!coarse_rhs[m - 1]) fail(CC_EINVAL, "null coarse right-hand side");
    const LevelHost& Lm = *p->lv[level];
    const int m = Lm.n, n0 = p->lv[0]->n;
    const long long m3 = cube(m);
    level_volfrac(p, level);
    if (p->net_cells < m3) {
      p->net_x = p->buf.alloc<float>(2 * m3);
      p->net_y = p->buf.alloc<float>(m3);
      p->net_cells = m3;
    }
    if (p->w64.nb < 1) alloc_work(p, p->w64, 1);
    fmg_alloc(p, 1);
    launch_zero_u64(p->d_norm, 1, p->stream);
    launch_maxabs(r, cube(n0), 1, p->d_norm, p->d_partial, p->stream);
    const double rn = read_norm(p);
    if (!std::isfinite(rn)) fail(CC_EINVAL, "non-finite right-hand side");
    const double inv = rn > 0 ? 1.0 / rn : 0.0;
    launch_net_features(n0, m, r, inv, p->volfrac[level], p->net_x, p->stream);
    HIPSYNC(p->stream);
    int rc = cc_net_forward(net, m, 1, p->net_x, p->net_y);
    if (rc != CC_OK) fail(rc, cc_last_error());
    launch_net_to_level(p->dev[level].st, p->net_y, rn / phi_scale, p->fmg_x[level], p->stream);
    fmg(p, p->w64, r, coarse_rhs, 0, phi, cycles, 1, p->fmg_rhs, p->fmg_x, level);
    HIPSYNC(p->stream);
  });
}

int cc_set_precision(cc_problem* p, int precision) {
  return guard([&] {
    if (!p) fail(CC_EINVAL, "null problem");
    if (precision != CC_FP64 && precision != CC_MIXED) fail(CC_EINVAL, "precision must be CC_FP64 or CC_MIXED");
    p->prm.precision = precision;
  });
}

int cc_solve_multi(int nprob, cc_problem* const* probs, const double* const* r, double* const* phi,
                   cc_solve_info* info) {
  if (nprob < 1 || !probs || !r || !phi) {
    set_last_error("bad argument");
    return CC_EINVAL;
  }
  for (int i = 0; i < nprob; ++i) {
    if (!probs[i] || !r[i] || !phi[i] || probs[i]->device < 0) {
      set_last_error("null or host-only problem in the list");
      return CC_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i] || probs[j]->stream == probs[i]->stream) {
        set_last_error("every problem needs its own handle and stream");
        return CC_EINVAL;
      }
  }
  std::vector<int> rc(nprob, CC_OK);
  std::vector<std::string> msg(nprob);
  std::vector<std::thread> th;
  for (int i = 0; i < nprob; ++i)
    th.emplace_back([&, i] {
      (void)hipSetDevice(probs[i]->device);
      rc[i] = cc_solve(probs[i], r[i], phi[i], info ? info + i : nullptr);
      if (rc[i] != CC_OK) msg[i] = cc_last_error();
    });
  for (auto& t : th) t.join();
  int worst = CC_OK;
  for (int i = 0; i < nprob; ++i)
    if (rc[i] != CC_OK && (worst == CC_OK || worst == CC_ENOCONV)) {
      worst = rc[i];
      set_last_error("problem " + std::to_string(i) + ": " + msg[i]);
    }
  return worst;
}

namespace {

// One problem of a lockstep multi-problem iteration.
struct MultiSlot {
  cc_problem* P = nullptr;
  const double* r = nullptr;
  double* phi = nullptr;
  bool mixed = false;
  std::vector<double> rn;
  std::vector<SolveRec> rec;
  bool done = false;
  int it = 0;
  hipGraphExec_t gexec() const { return mixed ? P->w32.gexec : P->w64.gexec; }
  unsigned long long* norm() const { return mixed ? P->w32.norm : P->w64.norm; }
};



}  // namespace

int cc_solve_multi_graph(int nprob, cc_problem* const* probs, const double* const* r, double* const* phi,
                         cc_solve_info* info) {
  int all_conv = 1;
  int rc = guard([&] {
    if (nprob < 1 || !probs || !r || !phi) fail(CC_EINVAL, "bad argument");
    std::vector<MultiSlot> S(nprob);
    for (int i = 0; i < nprob; ++i) {
      if (!probs[i] || !r[i] || !phi[i] || probs[i]->device < 0) fail(CC_EINVAL, "null or host-only problem in the list");
      if (probs[i]->device != probs[0]->device) fail(CC_EINVAL, "every problem must live on one device");
      if (probs[i]->prm.krylov > 0) fail(CC_EINVAL, "the lockstep iteration is the plain multigrid iteration (krylov 0)");
      for (int j = 0; j < i; ++j)
        if (probs[j] == probs[i]) fail(CC_EINVAL, "a problem appears twice in the list");
      S[i].P = probs[i];
      S[i].r = r[i];
      S[i].phi = phi[i];
      S[i].mixed = probs[i]->prm.precision == CC_MIXED;
    }
    HIPCHK(hipSetDevice(probs[0]->device));
    const double t0 = now_s();
    // each problem's prologue and captured outer step, on its own stream
    for (MultiSlot& m : S) {
      if (m.mixed) {
        if (m.P->w32.nb < 1) alloc_work(m.P, m.P->w32, 1);
        m.done = loop_prologue<float>(m.P, m.P->w32, m.r, m.phi, 1, m.rn, m.rec);
        if (!m.done) ensure_graph<float>(m.P, m.P->w32, m.r, m.phi, 1);
      } else {
        m.done = loop_prologue<double>(m.P, m.P->w64, m.r, m.phi, 1, m.rn, m.rec);
        if (!m.done) ensure_graph<double>(m.P, m.P->w64, m.r, m.phi, 1);
      }
      HIPSYNC(m.P->stream);
    }
    // every iteration: each unconverged problem's captured outer step launched
    // on its own stream from this one host thread (the problems' kernels
    // overlap on the device), then all their residual norms read back
    std::vector<int> act;
    std::vector<unsigned long long> bits(nprob);
    while (true) {
      act.clear();
      for (int i = 0; i < nprob; ++i)
        if (!S[i].done && S[i].it < S[i].P->prm.max_iter) act.push_back(i);
      if (act.empty()) break;
      for (int i : act) HIPCHK(hipGraphLaunch(S[i].gexec(), S[i].P->stream));
      for (int i : act)
        HIPCHK(hipMemcpyAsync(&bits[i], S[i].norm(), sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              S[i].P->stream));
      for (int i : act) HIPSYNC(S[i].P->stream);
      for (int i : act) {
        double v;
        std::memcpy(&v, &bits[i], sizeof(double));
        ++S[i].it;
        S[i].done = update_rec(S[i].P, S[i].rn, std::vector<double>{v}, S[i].rec, false);
      }
    }
    for (MultiSlot& m : S) {
      DevLevel& D0 = m.P->dev[0];
      launch_copy_pairs<double>(D0.n_absorbed, D0.absorbed, m.phi, cube(D0.st.n), 1, m.P->stream);
      HIPSYNC(m.P->stream);
    }
    const double dt = now_s() - t0;
    for (int i = 0; i < nprob; ++i) {
      if (info) fill_info(S[i].rec[0], dt, info + i);
      if (!(S[i].rec[0].rel < S[i].P->prm.tol)) all_conv = 0;
    }
  });
  if (rc == CC_OK && !all_conv) {
    set_last_error("max_iter reached before tol on at least one problem");
    return CC_ENOCONV;
  }
  return rc;
}

int cc_set_overlap(cc_problem* p, int on) {
  return guard([&] {
    if (!p) fail(CC_EINVAL, "null problem");
    need_device(p);
    if (on != 0 && on != 1) fail(CC_EINVAL, "on must be 0 or 1");
    HIPCHK(hipSetDevice(p->device));
    HIPSYNC(p->stream);
    p->overlap = on;
    // captured iterations hold the old launch structure
    p->w64.drop_graph();
    p->w32.drop_graph();
    p->wb64.drop_graph();
    p->wb32.drop_graph();
  });
}

int cc_set_krylov(cc_problem* p, int krylov) {
  return guard([&] {
    if (!p) fail(CC_EINVAL, "null problem");
    if (krylov < 0 || krylov > 64) fail(CC_EINVAL, "krylov must lie in [0, 64]");
    p->prm.krylov = krylov;
  });
}

int cc_set_lu_schedule(cc_problem* p, int level, int entries_per_lane, int subtree, int waves_cap) {
  return guard([&] {
    if (!p) fail(CC_EINVAL, "null problem");
    need_device(p);
    if (level < 0 || level >= (int)p->dev.size()) fail(CC_EINVAL, "bad level");
    if (entries_per_lane != 2 && entries_per_lane != 4 && entries_per_lane != 8 && entries_per_lane != 16 &&
        entries_per_lane != 32)
      fail(CC_EINVAL, "entries_per_lane must be 2, 4, 8, 16 or 32");
    if (subtree < 0 || subtree > 2) fail(CC_EINVAL, "subtree must be 0, 1 or 2");
    if (waves_cap != 0 && waves_cap < 4) fail(CC_EINVAL, "waves_cap must be 0 or at least 4");
    HIPCHK(hipSetDevice(p->device));
    HIPSYNC(p->stream);  // no launch in flight reads the old task lists
    DevLevel& D = p->dev[level];
    DevBuf nb;
    DevLU L = D.lu;
    make_schedule(p->lu[level], L, (double)entries_per_lane, nb);
    if (subtree == 1 && L.sub.nsub == 0) {
      nb.release();
      fail(CC_EINVAL, "this factorization has no subtree launch (cc_level_info.lu_subtrees is 0)");
    }
    L.sub_on = subtree == 1;
    L.flow_on = subtree == 2;
    if (L.flow_on) {
      make_flow(p->lu[level], L, (double)entries_per_lane, nb);
      L.flow.max_waves = waves_cap;
    }
    L.epl = entries_per_lane;
    L.wcap = waves_cap == 0 ? (1 << 30) : waves_cap;
    for (LuTasks& T : L.tasks) T.wcap = L.wcap;
    D.sched.release();
    D.sched = std::move(nb);
    D.lu = L;
    // captured iterations hold the old task lists
    p->w64.drop_graph();
    p->w32.drop_graph();
    p->wb64.drop_graph();
    p->wb32.drop_graph();
  });
}

int cc_set_stencil_schedule(cc_problem* p, int level, int march, int planes) {
  return guard([&] {
    if (!p) fail(CC_EINVAL, "null problem");
    need_device(p);
    const int nl = (int)p->dev.size();
    if (level < -1 || level >= nl) fail(CC_EINVAL, "bad level");
    if (march < -1 || march > 2) fail(CC_EINVAL, "march must be -1, 0, 1 or 2");
    for (int m = (level < 0 ? 0 : level); m < (level < 0 ? nl : level + 1); ++m)
      if (planes < 0 || planes > p->dev[m].st.n) fail(CC_EINVAL, "planes must lie in [0, n] of the level");
    HIPCHK(hipSetDevice(p->device));
    HIPSYNC(p->stream);
    for (int m = (level < 0 ? 0 : level); m < (level < 0 ? nl : level + 1); ++m) {
      StencilLevel& S = p->dev[m].st;
      S.march = march < 0 ? p->dev[m].tuned_march : march;
      S.kz = planes == 0 ? p->dev[m].tuned_kz : planes;
    }
    // captured iterations hold the old launch shapes
    p->w64.drop_graph();
    p->w32.drop_graph();
    p->wb64.drop_graph();
    p->wb32.drop_graph();
  });
}

int cc_get_stencil_schedule(const cc_problem* p, int level, int* march, int* planes) {
  return guard([&] {
    if (!p || !march || !planes) fail(CC_EINVAL, "null argument");
    need_device(p);
    if (level < 0 || level >= (int)p->dev.size()) fail(CC_EINVAL, "bad level");
    *march = p->dev[level].st.march;
    *planes = p->dev[level].st.kz;
  });
}

int cc_solve_batched(cc_problem* p, int nrhs, const double* r, double* phi, cc_solve_info* info) {
  int conv = 1;
  int rc = guard([&] {
    if (!p || !r || !phi || nrhs < 1) fail(CC_EINVAL, "bad argument");
    need_device(p);
    const long long n3 = cube(p->dev[0].st.n);
    const int cap = std::min(nrhs, CC_BATCH_MAX);
    const bool mixed = p->prm.precision == CC_MIXED;
    if (p->prm.krylov <= 0 && (mixed ? p->wb32.nb < cap : p->wb64.nb < cap)) {
      if (mixed)
        alloc_work(p, p->wb32, cap);
      else
        alloc_work(p, p->wb64, cap);
    }
    if (p->prm.krylov > 0) {  // Krylov acceleration: one right-hand side at a time
      for (int b = 0; b < nrhs; ++b) {
        double t0 = now_s();
        SolveRec rc;
        gmres_loop(p, r + b * n3, phi + b * n3, rc);
        if (info) fill_info(rc, now_s() - t0, info + b);
        if (!(rc.rel < p->prm.tol)) conv = 0;
      }
      return;
    }
    for (int b0 = 0; b0 < nrhs; b0 += CC_BATCH_MAX) {
      const int nb = std::min(CC_BATCH_MAX, nrhs - b0);
      double t0 = now_s();
      std::vector<SolveRec> rec;
      if (mixed)
        solve_loop<float>(p, p->wb32, r + b0 * n3, phi + b0 * n3, nb, rec);
      else
        solve_loop<double>(p, p->wb64, r + b0 * n3, phi + b0 * n3, nb, rec);
      double dt = now_s() - t0;
      for (int b = 0; b < nb; ++b) {
        if (info) fill_info(rec[b], dt, info + b0 + b);
        if (!(rec[b].rel < p->prm.tol)) conv = 0;
      }
    }
  });
  if (rc == CC_OK && !conv) {
    set_last_error("max_iter reached before tol for some right-hand side");
    return CC_ENOCONV;
  }
  return rc;
}

// Algorithmic bytes of one LU-correction sweep pair (forward + backward) of a
// level with values of `vb` bytes: every stored factor entry once, the
// right-hand side, intermediate and solution vectors, index lists and the
// scatter to the grid.
static double lu_sweep_bytes(const SupernodalLU& F, double vb) {
  double b = 0.0;
  for (const SnNode& nd : F.nodes) {
    const double p = nd.p, q = nd.q;
    b += vb * (p * p + 2.0 * p * q);          // M (both triangles), V, W
    b += vb * (2.0 * p) + (vb * 2.0 + 4.0) * q;  // forward: y_F, z_F; y_U update, Uf
    b += vb * (3.0 * p) + (vb + 4.0) * q + 4.0 * p + 8.0 * p;  // backward: z_F, x_F, x_U, U, var_cell, out
  }
  return b;
}

int cc_time_kernel(cc_problem* p, int which, int reps, double* ms, double* bytes) {
  return guard([&] {
    if (!p || !ms || reps <= 0) fail(CC_EINVAL, "bad argument");
    need_device(p);
    DevLevel& D = p->dev[0];
    const long long n3 = cube(D.st.n);
    if ((which == CC_TIME_SMO1_F32 || which == CC_TIME_LU_F32) && p->w32.nb < 1) alloc_work(p, p->w32, 1);
    std::function<void()> launch;
    double by = 0.0;
    double* x0 = p->e0;
    double* x1 = D.et;
    switch (which) {
      case CC_TIME_SMO1:
        launch = [&] {
          launch_smo1<double>(D.st, p->prm.omega, p->s0, x0, x1, 1, p->stream);
          std::swap(x0, x1);
        };
        by = 25.0 * n3;
        break;
      case CC_TIME_SMO1_F32: {
        float* a = p->w32.e[0];
        float* b = p->w32.et[0];
        const float* s = p->w32.s[0];
        launch = [&p, &D, a, b, s]() mutable {
          launch_smo1<float>(D.st, p->prm.omega, s, a, b, 1, p->stream);
          std::swap(a, b);
        };
        by = 13.0 * n3;
        break;
      }
      case CC_TIME_LU:
      case CC_TIME_LU_F32: {
        if ((int)p->dev.size() < 2) fail(CC_EINVAL, "no LU-correction on a one-level problem");
        if (which == CC_TIME_LU) {
          launch = [&] {
            lu_sweeps<double, double>(p->stream, D.lu, D.lu.d, D.et, n3, 1);
          };
          by = lu_sweep_bytes(p->lu[0], 8.0);
        } else {
          const LuDev F = p->w32.lu[0];
          float* out = p->w32.et[0];
          launch = [&p, &D, F, out] {
            lu_sweeps<float, float>(p->stream, D.lu, F, out, cube(D.st.n), 1);
          };
          by = lu_sweep_bytes(p->lu[0], 4.0);
        }
        break;
      }
      case CC_TIME_COPY:
        launch = [&] { launch_copy(n3, p->s0, p->e0, p->stream); };
        by = 16.0 * n3;
        break;
      default:
        fail(CC_EINVAL, "unknown kernel id");
    }
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    launch();
    HIPCHK(hipEventRecord(a, p->stream));
    for (int i = 0; i < reps; ++i) launch();
    HIPCHK(hipEventRecord(b, p->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(b));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, a, b));
    flow_check(p);
    *ms = t / reps;
    if (bytes) *bytes = by;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  });
}

void cc_destroy(cc_problem* p) {
  if (!p) return;
  if (p->device >= 0) {
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->stream2) (void)hipStreamSynchronize(p->stream2);
    p->w64.drop_graph();
    for (DevLevel& d : p->dev) d.sched.release();
    p->kr.own.release();
    p->w32.release();
    p->wb64.release();
    p->wb32.release();
    p->buf.release();
    if (p->stream2) (void)hipStreamDestroy(p->stream2);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
  }
  delete p;
}

}  // extern "C"
