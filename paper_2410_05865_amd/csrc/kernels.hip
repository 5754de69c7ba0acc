// Device kernels of the multigrid solve (Sec. 5.3) for gfx950: the cell-averaged
// fourth-order stencil with wall ghosts (Sec. 2.3) used by SMO-1, residuals and
// restriction, piecewise-constant prolongation, FV-PLG rows, the level-by-level
// supernodal triangular solves of the LU-correction and bottom solver, max-norm
// reductions and right-hand-side cell averages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <stdexcept>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "quadrature.hpp"

namespace cc {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// max that propagates NaN (fmax drops it): a norm of data holding a NaN is NaN,
// so the callers' finiteness checks see it
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, kWave));
  return v;
}

// Workgroup reductions (blockDim.x a multiple of 64, at most 1024); the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[16];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) t += part[i];
  return t;
}
__device__ __forceinline__ double block_max(double v) {
  __shared__ double part[16];
  v = wave_max(v);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) part[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) t = nan_max(t, part[i]);
  return t;
}

// One axis of the assembled regular row (times 12 h^2): the 5-point
// fourth-order stencil, with the ghost-substituted forms in the two cell layers
// next to a Dirichlet (bc 0), Neumann (bc 1) or Robin (bc 2: the level's
// assembled rows L.rob) wall.  x(d) is the operand at offset d (-3..3) along
// axis `ax`; adds the diagonal to diag.
template <class T, class X>
__device__ __forceinline__ T axis_op_at(X x, int t, int n, const StencilLevel& L, int ax, T& diag) {
  const int blo = L.bc[2 * ax], bhi = L.bc[2 * ax + 1];
  if (t >= 2 && t <= n - 3) {
    diag += T(-30.0);
    return -x(-2) + T(16.0) * x(-1) - T(30.0) * x(0) + T(16.0) * x(1) - x(2);
  }
  if (t == n - 1) {
    if (bhi == 2) {
      const double* r = L.rob[2 * ax + 1][0];
      diag += T(r[0]);
      return T(r[0]) * x(0) + T(r[1]) * x(-1) + T(r[2]) * x(-2) + T(r[3]) * x(-3);
    }
    if (bhi == 0) {
      diag += T(-1087.0 / 12.0);
      return (T(21.0) * x(-3) - T(139.0) * x(-2) + T(545.0) * x(-1) - T(1087.0) * x(0)) / T(12.0);
    }
    diag += T(-14.5);
    return T(0.1) * x(-3) - T(1.5) * x(-2) + T(15.9) * x(-1) - T(14.5) * x(0);
  }
  if (t == n - 2) {
    if (bhi == 2) {
      const double* r = L.rob[2 * ax + 1][1];
      diag += T(r[1]);
      return T(r[0]) * x(1) + T(r[1]) * x(0) + T(r[2]) * x(-1) + T(r[3]) * x(-2);
    }
    if (bhi == 0) {
      diag += T(-403.0 / 12.0);
      return (T(-15.0) * x(-2) + T(209.0) * x(-1) - T(403.0) * x(0) + T(269.0) * x(1)) / T(12.0);
    }
    diag += T(-30.9);
    return T(-1.1) * x(-2) + T(16.5) * x(-1) - T(30.9) * x(0) + T(15.5) * x(1);
  }
  if (t == 0) {
    if (blo == 2) {
      const double* r = L.rob[2 * ax][0];
      diag += T(r[0]);
      return T(r[0]) * x(0) + T(r[1]) * x(1) + T(r[2]) * x(2) + T(r[3]) * x(3);
    }
    if (blo == 0) {
      diag += T(-1087.0 / 12.0);
      return (T(21.0) * x(3) - T(139.0) * x(2) + T(545.0) * x(1) - T(1087.0) * x(0)) / T(12.0);
    }
    diag += T(-14.5);
    return T(0.1) * x(3) - T(1.5) * x(2) + T(15.9) * x(1) - T(14.5) * x(0);
  }
  // t == 1
  if (blo == 2) {
    const double* r = L.rob[2 * ax][1];
    diag += T(r[1]);
    return T(r[0]) * x(-1) + T(r[1]) * x(0) + T(r[2]) * x(1) + T(r[3]) * x(2);
  }
  if (blo == 0) {
    diag += T(-403.0 / 12.0);
    return (T(-15.0) * x(2) + T(209.0) * x(1) - T(403.0) * x(0) + T(269.0) * x(-1)) / T(12.0);
  }
  diag += T(-30.9);
  return T(-1.1) * x(2) + T(16.5) * x(1) - T(30.9) * x(0) + T(15.5) * x(-1);
}

// The same axis with the operand read from x at stride s around cell c.
template <class T>
__device__ __forceinline__ T axis_op(const T* __restrict__ x, long c, long s, int t, int n, const StencilLevel& L,
                                     int ax, T& diag) {
  return axis_op_at<T>([&](int d) { return x[c + d * s]; }, t, n, L, ax, diag);
}

// (L x)_c * 12 h^2 for a phi_1 cell and its diagonal.
template <class T>
__device__ __forceinline__ T regular_row(const StencilLevel& L, const T* __restrict__ x, int i, int j, int k,
                                         long c, T& diag) {
  const int n = L.n;
  const long nn = (long)n * n;
  diag = T(0);
  T a = axis_op<T>(x, c, 1, i, n, L, 0, diag);
  a += axis_op<T>(x, c, n, j, n, L, 1, diag);
  a += axis_op<T>(x, c, nn, k, n, L, 2, diag);
  return a;
}

// Streaming accesses of the stencil kernels (arrays read or written once): in
// FP64 they bypass the caches, which then keep the stencil operand's
// neighbour planes (measured faster); in FP32 plain accesses measured faster.
template <class T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr (sizeof(T) == 8)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <class T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  if constexpr (sizeof(T) == 8)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// 1D grid over 64 x 4 x 1 cell tiles, z fastest: concurrently resident blocks
// work on a narrow range of (x, y) columns, so the +-2 z-neighbour planes are
// re-read from cache (measured faster than x- or y-fastest orders).  The batch
// index is blockIdx.y.
__device__ __forceinline__ void tile_ijk(int n, int& i, int& j, int& k) {
  const int b = blockIdx.x;
  k = b % n;
  const int r = b / n;
  const int ny = (n + 3) / 4;
  j = (r % ny) * 4 + threadIdx.y;
  i = (r / ny) * 64 + threadIdx.x;
}
__device__ __forceinline__ long long batch_off(int n) { return (long long)blockIdx.y * n * n * n; }

template <class T, bool Far = false>
__global__ void k_smo1(StencilLevel L, T omega, const T* __restrict__ s, const T* __restrict__ ein,
                       T* __restrict__ eout) {
  const int n = L.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  const long long o = batch_off(n);
  s += o;
  ein += o;
  eout += o;
  long c = i + (long)n * (j + (long)n * k);
  if (Far && L.zone[c]) return;
  T v = ein[c];
  if (L.type[c] == 1) {
    T diag;
    const T inv = T(L.inv12h2);
    T a = regular_row<T>(L, ein, i, j, k, c, diag);
    v += omega * (ld_stream(s + c) - a * inv) / (diag * inv);
  }
  st_stream(v, eout + c);
}

// SMO-1 on a list of phi_1 cells (the near sweep), one thread each, the
// arithmetic of k_smo1.
template <class T>
__global__ void k_smo1_list(StencilLevel L, T omega, const T* __restrict__ s, const T* __restrict__ ein,
                            T* __restrict__ eout, const int* __restrict__ cells, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int n = L.n;
  const long long o = batch_off(n);
  s += o;
  ein += o;
  eout += o;
  const long c = cells[t];
  const int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((long)n * n));
  T v = ein[c];
  T diag;
  const T inv = T(L.inv12h2);
  T a = regular_row<T>(L, ein, i, j, k, c, diag);
  v += omega * (ld_stream(s + c) - a * inv) / (diag * inv);
  st_stream(v, eout + c);
}

// The regular-row kernels marching in z: a workgroup takes a 64 x 4 cell tile
// of (x, y) columns through kz consecutive planes, one wavefront per x row.
// Each thread keeps its column's operand at planes k-3 .. k+3 in registers
// (one new plane loaded per step).  The workgroup shares the current plane of
// its tile and of the 2 rows on either side (8 rows; the tile rows with their
// 3 x-halo cells) through LDS for the x- and y-neighbours, double-buffered by
// plane parity: one workgroup barrier per plane orders the writes of a plane
// before its reads, and the reads of a plane before the writes two planes
// later.  Per plane each thread loads its column's value 3 planes ahead, the
// cell type and the right-hand side, and one value of the 4 y-halo rows (row
// j0 - 2 + w for wavefront w < 2, j0 + 2 + w for w >= 2); lanes 0 .. 5 also
// load the x-halo; the y-neighbours at +-3 (wall rows only) come from memory.
// The loads of plane k+1 are in flight while plane k is computed.  All loads
// are unconditional at clamped addresses (a clamped value is never used: every
// stencil reference of a cell in the grid stays in the grid).  About 4 vector
// memory instructions per cell against 15 for the one-cell-per-thread kernels,
// in the same arithmetic order (identical results).
//   kMarchSmo:      eout = e + omega (b - A e) / D on phi_1 cells, e elsewhere
//   kMarchSmoFar:   the same, written only where zone is 0
//   kMarchResidual: eout = b - A e on phi_1 cells, 0 elsewhere
//   kMarchApply:    eout = A e on phi_1 cells, 0 elsewhere (b unused)
constexpr int kHalo = 3;
enum { kMarchSmo = 0, kMarchResidual = 1, kMarchApply = 2, kMarchSmoFar = 3 };
template <class T>
struct MarchPlane {
  T yh;        // this thread's y-halo row value
  T b;         // right-hand side
  T h;         // x-halo cell (lanes 0 .. 5)
  int type;
};
// Workgroups go to the 8 XCDs round-robin (workgroup w to XCD w mod 8).  The
// XCD-aware order gives XCD x one contiguous range of tiles, in order: the
// z-blocks of a column then follow each other on one XCD (the 3 halo planes
// each shares with the next one come from that XCD's L2) and neighbouring
// columns run there at the same time (the y-halo rows).  A bijection of
// [0, T): XCD x receives q + (x < T mod 8) workgroups, q = T / 8.
__device__ __forceinline__ int xcd_tile(int w, int T) {
  const int q = T / 8, rem = T % 8, x = w % 8;
  return x * q + min(x, rem) + w / 8;
}
template <class T, int Mode>
__device__ __forceinline__ void march_body(const StencilLevel& L, T omega, const T* __restrict__ bv,
                                           const T* __restrict__ ein, T* __restrict__ eout, int kz) {
  constexpr int kW = 64 + 2 * kHalo;
  __shared__ T pl[2][8][kW];
  const int n = L.n;
  const int nzb = (n + kz - 1) / kz;
  int blk = L.march == 2 ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  const int zb = blk % nzb;
  blk /= nzb;
  const int ny = (n + 3) / 4;
  const int l = threadIdx.x, w = threadIdx.y;
  const int j0 = (blk % ny) * 4;
  const int j = j0 + w;
  const int i0 = (blk / ny) * 64;
  const int i = i0 + l;
  const bool valid = i < n && j < n;
  const long long o = batch_off(n);
  if constexpr (Mode != kMarchApply) bv += o;
  ein += o;
  eout += o;
  const long nn = (long)n * n;
  const int ic = min(i, n - 1), jc = min(j, n - 1);
  const long col = ic + (long)n * jc;
  // LDS rows: 0, 1 hold j0 - 2, j0 - 1; 2 .. 5 the tile; 6, 7 hold j0 + 4, j0 + 5
  const int trow = 2 + w;
  const int hrow = w < 2 ? w : w + 4;
  const long hycol = ic + (long)n * min(max(j0 + hrow - 2, 0), n - 1);
  // lanes 0..2 hold x = i0-3 .. i0-1, lanes 3..5 x = i0+64 .. i0+66, stored at
  // column x - i0 + 3
  const int hl = l < kHalo ? l : l + 64;
  const long hcol = min(max(i0 + hl - kHalo, 0), n - 1) + (long)n * jc;
  const int k0 = zb * kz, k1 = min(k0 + kz, n);
  auto load = [&](int kp) {
    MarchPlane<T> P;
    const long po = kp * nn;
    P.yh = ein[hycol + po];
    P.type = L.type[col + po];
    if constexpr (Mode != kMarchApply)
      P.b = ld_stream(bv + col + po);
    else
      P.b = T(0);
    P.h = l < 2 * kHalo ? ein[hcol + po] : T(0);
    return P;
  };
  T q[2 * kHalo + 1];
#pragma unroll
  for (int d = -kHalo; d < kHalo; ++d) q[kHalo + d] = ein[col + min(max(k0 + d, 0), n - 1) * nn];
  MarchPlane<T> cur = load(k0);
  const T inv = T(L.inv12h2);
  // Planes in chunks of 8 with the steps unrolled: the register queue and the
  // plane buffers then rotate by renaming, not by moves (a move out of a
  // register whose load is in flight waits for that load), and the LDS buffer
  // of step u is the constant u & 1.  The guard is uniform over the
  // workgroup, so every wavefront takes the same barriers.
  for (int kc = k0; kc < k1; kc += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kc + u;
      if (k < k1) {
        T(*P)[kW] = pl[u & 1];
        q[2 * kHalo] = ein[col + min(k + kHalo, n - 1) * nn];
        const MarchPlane<T> nxt = load(min(k + 1, k1 - 1));
        const long c = col + k * nn;
        P[trow][kHalo + l] = q[kHalo];
        if (l < 2 * kHalo) P[trow][hl] = cur.h;
        P[hrow][kHalo + l] = cur.yh;
        __syncthreads();
        T v = (Mode == kMarchSmo || Mode == kMarchSmoFar) ? q[kHalo] : T(0);
        if (valid && cur.type == 1) {
          T diag = T(0);
          T a = axis_op_at<T>([&](int d) { return P[trow][kHalo + l + d]; }, i, n, L, 0, diag);
          a += axis_op_at<T>(
              [&](int d) {
                return d == 0 ? q[kHalo] : (d == -3 || d == 3) ? ein[c + d * (long)n] : P[trow + d][kHalo + l];
              },
              j, n, L, 1, diag);
          a += axis_op_at<T>([&](int d) { return q[kHalo + d]; }, k, n, L, 2, diag);
          if constexpr (Mode == kMarchSmo || Mode == kMarchSmoFar)
            v += omega * (cur.b - a * inv) / (diag * inv);
          else if constexpr (Mode == kMarchResidual)
            v = cur.b - a * inv;
          else
            v = a * inv;
        }
        if (valid && (Mode != kMarchSmoFar || L.zone[c] == 0)) st_stream(v, eout + c);
#pragma unroll
        for (int d = 0; d < 2 * kHalo; ++d) q[d] = q[d + 1];
        cur = nxt;
      }
    }
  }
}
template <class T>
__global__ __launch_bounds__(256) void k_smo1_z(StencilLevel L, T omega, const T* __restrict__ s,
                                                const T* __restrict__ ein, T* __restrict__ eout, int kz) {
  march_body<T, kMarchSmo>(L, omega, s, ein, eout, kz);
}
template <class T>
__global__ __launch_bounds__(256) void k_smo1_far_z(StencilLevel L, T omega, const T* __restrict__ s,
                                                    const T* __restrict__ ein, T* __restrict__ eout, int kz) {
  march_body<T, kMarchSmoFar>(L, omega, s, ein, eout, kz);
}
__global__ __launch_bounds__(256) void k_stencil_residual_z(StencilLevel L, const double* __restrict__ r,
                                                            const double* __restrict__ x, double* __restrict__ s,
                                                            int kz) {
  march_body<double, kMarchResidual>(L, 0.0, r, x, s, kz);
}
__global__ __launch_bounds__(256) void k_stencil_apply_z(StencilLevel L, const double* __restrict__ x,
                                                         double* __restrict__ y, int kz) {
  march_body<double, kMarchApply>(L, 0.0, nullptr, x, y, kz);
}

// Diagonal of the assembled regular row (times 12 h^2), summed over the axes in
// the order regular_row uses.
template <class T>
__device__ __forceinline__ T axis_diag(int t, int n, const StencilLevel& L, int ax) {
  const int blo = L.bc[2 * ax], bhi = L.bc[2 * ax + 1];
  if (t >= 2 && t <= n - 3) return T(-30.0);
  if (t == n - 1) return bhi == 2 ? T(L.rob[2 * ax + 1][0][0]) : bhi == 0 ? T(-1087.0 / 12.0) : T(-14.5);
  if (t == n - 2) return bhi == 2 ? T(L.rob[2 * ax + 1][1][1]) : bhi == 0 ? T(-403.0 / 12.0) : T(-30.9);
  if (t == 0) return blo == 2 ? T(L.rob[2 * ax][0][0]) : blo == 0 ? T(-1087.0 / 12.0) : T(-14.5);
  return blo == 2 ? T(L.rob[2 * ax][1][1]) : blo == 0 ? T(-403.0 / 12.0) : T(-30.9);
}

// The first SMO-1 sweep of a V-cycle level, from e = 0: e' = omega s / D on
// phi_1 cells, 0 elsewhere (the same arithmetic as k_smo1 with e = 0).
template <class T>
__global__ void k_smo1_first(StencilLevel L, T omega, const T* __restrict__ s, T* __restrict__ eout) {
  const int n = L.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  const long long o = batch_off(n);
  s += o;
  eout += o;
  long c = i + (long)n * (j + (long)n * k);
  T v = T(0);
  if (L.type[c] == 1) {
    T diag = T(0);
    diag += axis_diag<T>(i, n, L, 0);
    diag += axis_diag<T>(j, n, L, 1);
    diag += axis_diag<T>(k, n, L, 2);
    const T inv = T(L.inv12h2);
    v += omega * (ld_stream(s + c) - T(0) * inv) / (diag * inv);
  }
  st_stream(v, eout + c);
}

__global__ void k_stencil_residual(StencilLevel L, const double* __restrict__ r, const double* __restrict__ x,
                                   double* __restrict__ s, int apply) {
  const int n = L.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  const long long o = batch_off(n);
  x += o;
  s += o;
  if (!apply) r += o;
  long c = i + (long)n * (j + (long)n * k);
  double v = 0.0;
  if (L.type[c] == 1) {
    double diag;
    double a = regular_row<double>(L, x, i, j, k, c, diag) * L.inv12h2;
    v = apply ? a : __builtin_nontemporal_load(r + c) - a;
  }
  __builtin_nontemporal_store(v, s + c);
}

template <class T>
__device__ __forceinline__ const T* plg_vals(const PlgRows& P);
template <>
__device__ __forceinline__ const double* plg_vals<double>(const PlgRows& P) {
  return P.vals;
}
template <>
__device__ __forceinline__ const float* plg_vals<float>(const PlgRows& P) {
  return P.vals32;
}

// sum over the row's 35 entries of vals * x[cols] (entries whose bit is set in
// `skip` left out), kPlgLanes adjacent lanes per row: lane `sub` takes entries
// sub, sub + kPlgLanes, ...; its indices are loaded first, then its
// coefficients and gathered values, and the lanes' sums are added by
// shuffles (valid in every lane of the row's group).  Rows of one wavefront
// are consecutive, so each entry slot t is read coalesced across them.
constexpr int kPlgLanes = 4;
template <class T, class TX>
__device__ __forceinline__ T plg_dot(const PlgRows& P, const T* __restrict__ vals, const TX* __restrict__ x, int row,
                                     int sub, uint64_t skip) {
  constexpr int U = (35 + kPlgLanes - 1) / kPlgLanes;
  const long N2 = P.N2;
  int col[U];
#pragma unroll
  for (int u = 0; u < U; ++u) col[u] = P.cols[min(sub + u * kPlgLanes, 34) * N2 + row];
  T a = T(0);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = sub + u * kPlgLanes;
    const T v = vals[min(t, 34) * N2 + row] * T(x[col[u]]);
    if (t < 35 && !((skip >> t) & 1ull)) a += v;
  }
#pragma unroll
  for (int o = kPlgLanes / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
  return a;
}

// one row per kPlgLanes threads; rows past N2 take the last row's loads (the
// whole lane group alike) and store nothing
__global__ void k_plg_residual(PlgRows P, const double* __restrict__ r, const double* __restrict__ x,
                               double* __restrict__ s, int apply, long long stride) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row0 = (int)(tid / kPlgLanes), sub = (int)(tid % kPlgLanes);
  const int row = min(row0, P.N2 - 1);
  const long long o = (long long)blockIdx.y * stride;
  x += o;
  s += o;
  if (!apply) r += o;
  const double a = plg_dot<double, double>(P, P.vals, x, row, sub, 0ull);
  if (row0 < P.N2 && sub == 0) {
    int c = P.cell[row];
    s[c] = apply ? a : r[c] - a;
  }
}

// b_2 = s_2 - L21 e_1 of every FV-PLG row, written in factorization order
// (y[position * nb + batch]).
template <class T>
__global__ void k_plg_b2(PlgRows P, const T* __restrict__ s, const T* __restrict__ e, T* __restrict__ y,
                         long long stride) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row0 = (int)(tid / kPlgLanes), sub = (int)(tid % kPlgLanes);
  const int row = min(row0, P.N2 - 1);
  const int b = blockIdx.y, nb = gridDim.y;
  s += b * stride;
  e += b * stride;
  const T a = plg_dot<T, T>(P, plg_vals<T>(P), e, row, sub, P.phi2[row]);
  if (row0 < P.N2 && sub == 0) y[(long long)P.nd[row] * nb + b] = s[P.cell[row]] - a;
}

// coarse cell = 2^-3 sum over its 8 children of (s - L e) on phi_1 children
template <class T>
__global__ void k_restrict(StencilLevel F, StencilLevel C, const T* __restrict__ s, const T* __restrict__ e,
                           T* __restrict__ sc) {
  const int nc = C.n, nf = F.n;
  int I, J, K;
  tile_ijk(nc, I, J, K);
  if (I >= nc || J >= nc) return;
  const long long of = batch_off(nf);
  s += of;
  e += of;
  sc += batch_off(nc);
  long cc = I + (long)nc * (J + (long)nc * K);
  T acc = T(0);
  if (C.type[cc] != 0) {
    const T inv = T(F.inv12h2);
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
          long c = i + (long)nf * (j + (long)nf * k);
          if (F.type[c] != 1) continue;
          T diag;
          acc += ld_stream(s + c) - regular_row<T>(F, e, i, j, k, c, diag) * inv;
        }
  }
  st_stream(T(0.125) * acc, sc + cc);
}

template <class T>
__global__ void k_prolong_add(StencilLevel F, int nc, const T* __restrict__ ec, T* __restrict__ ef) {
  const int n = F.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  ef += batch_off(n);
  ec += batch_off(nc);
  long c = i + (long)n * (j + (long)n * k);
  if (F.type[c] == 1) ef[c] += ec[(i >> 1) + (long)nc * ((j >> 1) + (long)nc * (k >> 1))];
}

// Full multigrid transfers (Sec. 5, algorithm FMG).  Right-hand side:
// sc = 2^-3 sum of s over the 8 children that carry an unknown (type != 0);
// coarse cells without an unknown get 0.
__global__ void k_fmg_restrict(StencilLevel F, StencilLevel C, const double* __restrict__ s,
                               double* __restrict__ sc) {
  const int nc = C.n, nf = F.n;
  int I, J, K;
  tile_ijk(nc, I, J, K);
  if (I >= nc || J >= nc) return;
  const long cc = I + (long)nc * (J + (long)nc * K);
  s += batch_off(nf);
  sc += batch_off(nc);
  double acc = 0.0;
  if (C.type[cc] != 0) {
    double v[8];
    uint8_t t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long c = (2 * I + (q & 1)) + (long)nf * ((2 * J + ((q >> 1) & 1)) + (long)nf * (2 * K + (q >> 2)));
      v[q] = s[c];
      t[q] = F.type[c];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += t[q] != 0 ? v[q] : 0.0;
    acc *= 0.125;
  }
  sc[cc] = acc;
}

// Interpolation: trilinear in the coarse cell centres over the 8 coarse cells
// around each fine centre that lie in the box and carry an unknown, weights
// renormalised (0 if none); fine cells without an unknown get 0.
__global__ void k_fmg_prolong(StencilLevel F, StencilLevel C, const double* __restrict__ xc,
                              double* __restrict__ xf) {
  const int n = F.n, nc = C.n;
  int i, j, k;
  tile_ijk(n, i, j, k);
  if (i >= n || j >= n) return;
  const long c = i + (long)n * (j + (long)n * k);
  xc += batch_off(nc);
  xf += batch_off(n);
  double v = 0.0;
  if (F.type[c] != 0) {
    // fine centre (i + 1/2) h in coarse index units is i/2 - 1/4
    const int lo[3] = {(i & 1) ? i / 2 : i / 2 - 1, (j & 1) ? j / 2 : j / 2 - 1, (k & 1) ? k / 2 : k / 2 - 1};
    const double t[3] = {(i & 1) ? 0.25 : 0.75, (j & 1) ? 0.25 : 0.75, (k & 1) ? 0.25 : 0.75};
    double num = 0.0, den = 0.0;
    for (int dz = 0; dz < 2; ++dz) {
      const int kz = lo[2] + dz;
      if (kz < 0 || kz >= nc) continue;
      const double wz = dz ? t[2] : 1.0 - t[2];
      for (int dy = 0; dy < 2; ++dy) {
        const int jy = lo[1] + dy;
        if (jy < 0 || jy >= nc) continue;
        const double wy = dy ? t[1] : 1.0 - t[1];
        for (int dx = 0; dx < 2; ++dx) {
          const int ix = lo[0] + dx;
          if (ix < 0 || ix >= nc) continue;
          const long q = ix + (long)nc * (jy + (long)nc * kz);
          if (C.type[q] == 0) continue;
          const double w = (dx ? t[0] : 1.0 - t[0]) * wy * wz;
          num += w * xc[q];
          den += w;
        }
      }
    }
    v = den > 0.0 ? num / den : 0.0;
  }
  xf[c] = v;
}

template <class TS, class TY>
__global__ void k_gather(int n, const int* __restrict__ cell, const TS* __restrict__ src, long long stride,
                         TY* __restrict__ y) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y, nb = gridDim.y;
  if (v < n) y[(long long)v * nb + b] = TY(src[b * stride + cell[v]]);
}

// ---------------------------------------------------------------- factorizations
// Rows of every node are stored row-major; the node's equations are numbered
// in pivot order, so its right-hand side is contiguous.

template <class T>
struct LuArr;
template <>
struct LuArr<double> {
  __device__ static const double* M(const LuDev& F) { return F.M; }
  __device__ static const double* V(const LuDev& F) { return F.V; }
  __device__ static const double* W(const LuDev& F) { return F.W; }
  __device__ static double* y(const LuDev& F) { return F.y; }
  __device__ static double* z(const LuDev& F) { return F.z; }
  __device__ static double* x(const LuDev& F) { return F.x; }
};
template <>
struct LuArr<float> {
  __device__ static const float* M(const LuDev& F) { return F.M32; }
  __device__ static const float* V(const LuDev& F) { return F.V32; }
  __device__ static const float* W(const LuDev& F) { return F.W32; }
  __device__ static float* y(const LuDev& F) { return F.y32; }
  __device__ static float* z(const LuDev& F) { return F.z32; }
  __device__ static float* x(const LuDev& F) { return F.x32; }
};

// acc += sum_{j in [j0, j1), j = gl mod g} a[j] * b[j].  Entries are loaded K
// per lane per round, every load of a round issued before the first product,
// so a row of at most K g entries costs one memory round trip.  Indices past
// the row are clamped to its last entry (an in-bounds load) and their products
// dropped.
// Loads and stores of the work vectors that other tasks of the same launch
// write (C: the one-launch sweeps): relaxed agent-scope atomics, coherent
// across the XCDs without cache maintenance; plain accesses otherwise.
template <bool C, class T>
__device__ __forceinline__ T ld_c(const T* p) {
  if constexpr (C)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool C, class T>
__device__ __forceinline__ void st_c(T* p, T v) {
  if constexpr (C)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}
template <int K, class T, bool C = false>
__device__ __forceinline__ T lane_dot(const T* __restrict__ a, const T* __restrict__ b, int j0, int j1, int gl,
                                      int g) {
  T s0 = T(0), s1 = T(0);
  for (int jb = j0 + gl; jb < j1; jb += K * g) {
    T va[K], vb[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int j = min(jb + u * g, j1 - 1);
      va[u] = a[j];
      vb[u] = ld_c<C>(b + j);
    }
#pragma unroll
    for (int u = 0; u < K; u += 2) {
      if (jb + u * g < j1) s0 += va[u] * vb[u];
      if (jb + (u + 1) * g < j1) s1 += va[u + 1] * vb[u + 1];
    }
  }
  return s0 + s1;
}

// Single right-hand side: a task takes 64/g rows of one node, g lanes per row.
// A wavefront runs a strided sequence of tasks in pairs: the descriptors and
// first load rounds of both tasks are issued before any of their products are
// formed, so their memory latencies overlap.
// Indices are clamped in bounds (U and Uf end with one padding entry, every
// node has p >= 1) and products past a row's end are dropped.
struct TaskLanes {
  int g, gl, i;
  __device__ TaskLanes(const LuTask& t, int lane) {
    g = 1 << t.lg;
    gl = lane & (g - 1);
    i = t.row0 + (lane >> t.lg);
  }
};

// Forward: z_F = L11^-1 y_F on the node's rows, and y_U -= (L21 L11^-1) y_F
// accumulated atomically into the later equations.
template <int K, class T>
struct FwdRound {
  T va[K], vb[K];
  T yi;
  int dst;
};
template <class T>
__device__ __forceinline__ const T* fwd_row(const LuDev& F, const LuTask& t, int ii) {
  return ii < t.p ? LuArr<T>::M(F) + t.offM + (long)ii * t.p : LuArr<T>::V(F) + t.offVW + (long)(ii - t.p) * t.p;
}
template <int K, class T, bool C = false>
__device__ __forceinline__ void fwd_issue(const LuDev& F, const LuTask& t, int lane, FwdRound<K, T>& r) {
  const TaskLanes L(t, lane);
  const int p = t.p, q = t.q;
  const int ii = min(L.i, p + q - 1);
  const T* yF = LuArr<T>::y(F) + t.base;
  r.yi = ld_c<C>(yF + min(ii, p - 1));
  r.dst = F.Uf[t.offU + max(ii - p, 0)];
  const T* row = fwd_row<T>(F, t, ii);
  const int jend = L.i < p + q ? (ii < p ? ii : p) : 0;
  const int jmax = max(jend - 1, 0);
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int j = min(L.gl + u * L.g, jmax);
    r.va[u] = row[j];
    r.vb[u] = ld_c<C>(yF + j);
  }
}
template <int K, class T, bool C = false>
__device__ __forceinline__ void fwd_finish(const LuDev& F, const LuTask& t, int lane, const FwdRound<K, T>& r) {
  const TaskLanes L(t, lane);
  const int p = t.p, q = t.q;
  const bool valid = L.i < p + q;
  const int ii = min(L.i, p + q - 1);
  const int jend = valid ? (ii < p ? ii : p) : 0;
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int u = 0; u < K; u += 2) {
    if (L.gl + u * L.g < jend) s0 += r.va[u] * r.vb[u];
    if (L.gl + (u + 1) * L.g < jend) s1 += r.va[u + 1] * r.vb[u + 1];
  }
  T acc = s0 + s1;
  if (L.gl + K * L.g < jend)
    acc += lane_dot<K, T, C>(fwd_row<T>(F, t, ii), LuArr<T>::y(F) + t.base, K * L.g, jend, L.gl, L.g);
  for (int o = L.g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (valid && L.gl == 0) {
    if (L.i < p)
      LuArr<T>::z(F)[t.base + L.i] = acc + r.yi;
    else
      atomicAdd(&LuArr<T>::y(F)[r.dst], -acc);
  }
}
// tasks t0, t0 + stride, ... below t1, two at a time: both descriptors, then
// both tasks' first load rounds, are issued before the first product (a lone
// last task is issued alone)
template <int K, class T>
__device__ __forceinline__ void fwd_tasks(const LuDev& F, const LuTask* __restrict__ tasks, int t0, int t1,
                                          int stride, int lane) {
  for (int ti = t0; ti < t1; ti += 2 * stride) {
    const bool two = ti + stride < t1;
    const LuTask ta = tasks[ti];
    LuTask tb = ta;
    if (two) tb = tasks[ti + stride];
    FwdRound<K, T> ra, rb;
    fwd_issue<K, T>(F, ta, lane, ra);
    if (two) fwd_issue<K, T>(F, tb, lane, rb);
    __builtin_amdgcn_sched_barrier(0);  // every load of the pair ahead of the products
    fwd_finish<K, T>(F, ta, lane, ra);
    if (two) fwd_finish<K, T>(F, tb, lane, rb);
  }
}

// Backward: x_F = U11^-1 z_F - (U11^-1 U12) x_U, scattered to the grid array
// `out` through var_cell.  The issue stage loads the first K indices of U per
// lane with the first round of the U11 part; the finish stage loads their
// coefficients with the gathered x_U.
template <int K, class T>
struct BwdRound {
  T va[K], vb[K];
  int uu[K];
  int cell;
};
template <int K, class T>
__device__ __forceinline__ void bwd_issue(const LuDev& F, const LuTask& t, int lane, BwdRound<K, T>& r) {
  const TaskLanes L(t, lane);
  const int p = t.p, q = t.q;
  const int ii = min(L.i, p - 1);
  r.cell = F.var_cell[t.base + ii];
  const int* U = F.U + t.offU;
  const int qmax = max(q - 1, 0);
#pragma unroll
  for (int u = 0; u < K; ++u) r.uu[u] = U[min(L.gl + u * L.g, qmax)];
  const T* Mr = LuArr<T>::M(F) + t.offM + (long)ii * p;
  const T* z = LuArr<T>::z(F) + t.base;
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int j = min(ii + L.gl + u * L.g, p - 1);
    r.va[u] = Mr[j];
    r.vb[u] = z[j];
  }
}
template <int K, class T, class TO, bool C = false>
__device__ __forceinline__ void bwd_finish(const LuDev& F, const LuTask& t, int lane, const BwdRound<K, T>& r,
                                           TO* __restrict__ out) {
  const TaskLanes L(t, lane);
  const int p = t.p, q = t.q;
  const bool valid = L.i < p;
  const int ii = min(L.i, p - 1);
  const int jlo = valid ? ii : p;
  T* x = LuArr<T>::x(F);
  const T* Wr = LuArr<T>::W(F) + t.offVW + (long)ii * q;
  const int* U = F.U + t.offU;
  // coefficients and gathered values of the first round of U12
  T w[K], vx[K];
  const int qmax = max(q - 1, 0);
#pragma unroll
  for (int u = 0; u < K; ++u) {
    w[u] = Wr[min(L.gl + u * L.g, qmax)];
    vx[u] = ld_c<C>(x + r.uu[u]);
  }
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int u = 0; u < K; u += 2) {
    if (jlo + L.gl + u * L.g < p) s0 += r.va[u] * r.vb[u];
    if (jlo + L.gl + (u + 1) * L.g < p) s1 += r.va[u + 1] * r.vb[u + 1];
  }
  T acc = s0 + s1;
  if (jlo + L.gl + K * L.g < p)
    acc += lane_dot<K, T>(LuArr<T>::M(F) + t.offM + (long)ii * p, LuArr<T>::z(F) + t.base, jlo + K * L.g, p, L.gl,
                          L.g);
  const int qv = valid ? q : 0;
  s0 = T(0);
  s1 = T(0);
#pragma unroll
  for (int u = 0; u < K; u += 2) {
    if (L.gl + u * L.g < qv) s0 += w[u] * vx[u];
    if (L.gl + (u + 1) * L.g < qv) s1 += w[u + 1] * vx[u + 1];
  }
  for (int jb = L.gl + K * L.g; jb < qv; jb += K * L.g) {
    int uu[K];
#pragma unroll
    for (int u = 0; u < K; ++u) uu[u] = U[min(jb + u * L.g, q - 1)];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      w[u] = Wr[min(jb + u * L.g, q - 1)];
      vx[u] = ld_c<C>(x + uu[u]);
    }
#pragma unroll
    for (int u = 0; u < K; u += 2) {
      if (jb + u * L.g < q) s0 += w[u] * vx[u];
      if (jb + (u + 1) * L.g < q) s1 += w[u + 1] * vx[u + 1];
    }
  }
  acc -= s0 + s1;
  for (int o = L.g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (valid && L.gl == 0) {
    st_c<C>(x + t.base + L.i, acc);
    out[r.cell] = TO(acc);
  }
}
template <int K, class T, class TO>
__device__ __forceinline__ void bwd_tasks(const LuDev& F, const LuTask* __restrict__ tasks, int t0, int t1,
                                          int stride, int lane, TO* __restrict__ out) {
  for (int ti = t0; ti < t1; ti += 2 * stride) {
    const bool two = ti + stride < t1;
    const LuTask ta = tasks[ti];
    LuTask tb = ta;
    if (two) tb = tasks[ti + stride];
    BwdRound<K, T> ra, rb;
    bwd_issue<K, T>(F, ta, lane, ra);
    if (two) bwd_issue<K, T>(F, tb, lane, rb);
    __builtin_amdgcn_sched_barrier(0);  // every load of the pair ahead of the products
    bwd_finish<K, T, TO>(F, ta, lane, ra, out);
    if (two) bwd_finish<K, T, TO>(F, tb, lane, rb, out);
  }
}

// Several right-hand sides (nb <= 64): a task takes up to kMrRows rows of one
// node; lane b works on right-hand side b.  The rows' entries are read 64 at a
// time, coalesced, and broadcast lane by lane, so every factor entry is read
// once for all right-hand sides; vector values are loaded 16 at a time so that
// their latencies overlap.
__device__ __forceinline__ double lane_bcast(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int lane_bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

constexpr int kMrBlock = 16;

// acc[r] += sum over the chunk's jn entries of ch[r](lane jj) * vec(jj); vec(jj)
// is v[jj * nb] for lanes < nb.  Entries jj >= jn have ch == 0.
template <class T>
__device__ __forceinline__ void mr_chunk(const T (&ch)[kMrRows], const T* __restrict__ v, int nb, int jn, bool act,
                                         T (&acc)[kMrRows]) {
  for (int jb = 0; jb < jn; jb += kMrBlock) {
    T vv[kMrBlock];
#pragma unroll
    for (int u = 0; u < kMrBlock; ++u) vv[u] = (act && jb + u < jn) ? v[(long long)(jb + u) * nb] : T(0);
#pragma unroll
    for (int u = 0; u < kMrBlock; ++u)
#pragma unroll
      for (int r = 0; r < kMrRows; ++r) acc[r] += lane_bcast(ch[r], jb + u) * vv[u];
  }
}

template <class T>
__device__ __forceinline__ void fwd_task_mr(const LuDev& F, const LuTask& t, int lane, int nb) {
  const bool act = lane < nb;
  T* y = LuArr<T>::y(F);
  const int p = t.p, q = t.q, base = t.base;
  const T* M = LuArr<T>::M(F) + t.offM;
  const T* V = LuArr<T>::V(F) + t.offVW;
  const T* ptr[kMrRows];
  int end[kMrRows];
  T acc[kMrRows];
  int jmax = 0;
#pragma unroll
  for (int r = 0; r < kMrRows; ++r) {
    const int i = t.row0 + r;
    acc[r] = T(0);
    if (i < p) {
      ptr[r] = M + (long)i * p;
      end[r] = i;
    } else if (i < p + q) {
      ptr[r] = V + (long)(i - p) * p;
      end[r] = p;
    } else {
      ptr[r] = M;
      end[r] = 0;
    }
    jmax = max(jmax, end[r]);
  }
  for (int j0 = 0; j0 < jmax; j0 += kWave) {
    T ch[kMrRows];
#pragma unroll
    for (int r = 0; r < kMrRows; ++r) ch[r] = (j0 + lane < end[r]) ? ptr[r][j0 + lane] : T(0);
    mr_chunk<T>(ch, y + (long long)(base + j0) * nb + lane, nb, min(kWave, jmax - j0), act, acc);
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < kMrRows; ++r) {
      const int i = t.row0 + r;
      if (i < p)
        LuArr<T>::z(F)[(long long)(base + i) * nb + lane] = acc[r] + y[(long long)(base + i) * nb + lane];
      else if (i < p + q)
        atomicAdd(&y[(long long)F.Uf[t.offU + (i - p)] * nb + lane], -acc[r]);
    }
  }
}

template <class T, class TO>
__device__ __forceinline__ void bwd_task_mr(const LuDev& F, const LuTask& t, int lane, int nb, TO* __restrict__ out,
                                            long long ostride) {
  const bool act = lane < nb;
  const T* z = LuArr<T>::z(F);
  T* x = LuArr<T>::x(F);
  const int p = t.p, q = t.q, base = t.base;
  const T* M = LuArr<T>::M(F) + t.offM;
  const T* W = LuArr<T>::W(F) + t.offVW;
  const int* U = F.U + t.offU;
  T acc[kMrRows];
#pragma unroll
  for (int r = 0; r < kMrRows; ++r) acc[r] = T(0);
  // U11^-1 z_F: row i uses columns [i, p)
  for (int j0 = t.row0; j0 < p; j0 += kWave) {
    T ch[kMrRows];
    const int j = j0 + lane;
#pragma unroll
    for (int r = 0; r < kMrRows; ++r) {
      const int i = t.row0 + r;
      ch[r] = (i < p && j >= i && j < p) ? M[(long)i * p + j] : T(0);
    }
    mr_chunk<T>(ch, z + (long long)(base + j0) * nb + lane, nb, min(kWave, p - j0), act, acc);
  }
  // - (U11^-1 U12) x_U
  for (int j0 = 0; j0 < q; j0 += kWave) {
    T ch[kMrRows];
    const int j = j0 + lane;
    const int uj = (j < q) ? U[j] : 0;
#pragma unroll
    for (int r = 0; r < kMrRows; ++r) {
      const int i = t.row0 + r;
      ch[r] = (i < p && j < q) ? -W[(long)i * q + j] : T(0);
    }
    const int jn = min(kWave, q - j0);
    for (int jb = 0; jb < jn; jb += kMrBlock) {
      T vv[kMrBlock];
#pragma unroll
      for (int u = 0; u < kMrBlock; ++u) {
        const int uu = lane_bcast(uj, jb + u);
        vv[u] = (act && jb + u < jn) ? x[(long long)uu * nb + lane] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kMrBlock; ++u)
#pragma unroll
        for (int r = 0; r < kMrRows; ++r) acc[r] += lane_bcast(ch[r], jb + u) * vv[u];
    }
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < kMrRows; ++r) {
      const int i = t.row0 + r;
      if (i < p) {
        x[(long long)(base + i) * nb + lane] = acc[r];
        out[lane * ostride + F.var_cell[base + i]] = TO(acc[r]);
      }
    }
  }
}

// One height of the tree per launch.  Single right-hand side: each wavefront
// takes the tasks w, w + W, ... (W wavefronts in the grid) through the
// pipeline; several right-hand sides: one task per wavefront.
template <int K, class T>
__global__ void __launch_bounds__(256) k_lu_forward(LuDev F, const LuTask* __restrict__ tasks, int ntasks, int nb) {
  const int w = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nw = gridDim.x * (blockDim.x / kWave);
  if (nb == 1) {
    fwd_tasks<K, T>(F, tasks, w, ntasks, nw, threadIdx.x % kWave);
  } else if (w < ntasks) {
    const LuTask t = tasks[w];
    fwd_task_mr<T>(F, t, threadIdx.x % kWave, nb);
  }
}
template <int K, class T, class TO>
__global__ void __launch_bounds__(256) k_lu_backward(LuDev F, const LuTask* __restrict__ tasks, int ntasks, int nb,
                                                     TO* __restrict__ out, long long ostride) {
  const int w = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nw = gridDim.x * (blockDim.x / kWave);
  if (nb == 1) {
    bwd_tasks<K, T, TO>(F, tasks, w, ntasks, nw, threadIdx.x % kWave, out);
  } else if (w < ntasks) {
    const LuTask t = tasks[w];
    bwd_task_mr<T, TO>(F, t, threadIdx.x % kWave, nb, out, ostride);
  }
}

// Both sweeps of an LU solve as one launch each (lu_flow.hpp).  The unit of
// the protocol is a wavefront, and the protocol's control flow is uniform over
// it: every lane takes part in the ticket and completion atomics (lane 0 adds
// the batch or 1, the others 0) and every value that steers the loop (ticket,
// counts, error word) is read through readfirstlane, so the loop and its
// waits branch on scalars.  (A lane-0-only ticket and signal let the compiler
// route lanes 1..63 past the ticket back to the broadcast of lane 0's register
// while lane 0 was inactive, where they re-ran task 0 for ever.)  Polls are
// relaxed agent-scope loads, which read the counter at the coherence point.
// The data the tasks of one launch pass to each other are accessed only by
// coherent agent-scope atomics (ld_c, st_c, atomicAdd), so the fences need no
// cache maintenance: the writer waits for its own accesses before it raises
// its count, and the reader issues its loads after its poll saw the count
// (the host model states the same order as a release increment and an
// acquire load).
struct DevSync {
  static __device__ int lane0() { return (threadIdx.x & (kWave - 1)) == 0 ? 1 : 0; }
  static __device__ int next_ticket(int* t, int n) {
    const int v = __hip_atomic_fetch_add(t, lane0() * n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_amdgcn_readfirstlane(v);
  }
  static __device__ int load_acquire(const int* p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  static __device__ int load_relaxed(const int* p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  static __device__ void set_err(int* p) { __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
  static __device__ long long now() { return wall_clock64(); }
  // about 0.2 us between polls: waiting wavefronts leave the memory system
  // to the working ones
  static __device__ void pause() { __builtin_amdgcn_s_sleep(8); }
  static __device__ void acquire_fence() {}
  static __device__ void release_fence() { __builtin_amdgcn_s_waitcnt(0); }
  static __device__ void signal(int* p) {
    __hip_atomic_fetch_add(p, lane0(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
template <int K, class T>
__global__ void __launch_bounds__(256) k_lu_forward_flow(LuDev F, const LuTask* __restrict__ tasks, FlowGraph G,
                                                         long long limit) {
  const int lane = threadIdx.x & (kWave - 1);
  flow_run<DevSync>(G, limit, [&](int t) {
    const LuTask tk = tasks[t];
    FwdRound<K, T> r;
    fwd_issue<K, T, true>(F, tk, lane, r);
    fwd_finish<K, T, true>(F, tk, lane, r);
  });
}
template <int K, class T, class TO>
__global__ void __launch_bounds__(256) k_lu_backward_flow(LuDev F, const LuTask* __restrict__ tasks, FlowGraph G,
                                                          long long limit, TO* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  flow_run<DevSync>(G, limit, [&](int t) {
    const LuTask tk = tasks[t];
    BwdRound<K, T> r;
    bwd_issue<K, T>(F, tk, lane, r);
    bwd_finish<K, T, TO, true>(F, tk, lane, r, out);
  });
}

// The lower heights of the tree in one launch: workgroup s takes subtree s
// through all its heights (levels lptr[s] .. lptr[s+1] of the list, each a
// range of tasks), its kSubWaves wavefronts sharing each height's tasks, with a
// workgroup barrier between heights (a subtree's values are written and read
// only by its workgroup; contributions to ancestors above the cut are device
// atomics read by later launches); nothing waits on another workgroup.
constexpr int kSubWaves = 8;  // wavefronts per subtree workgroup

template <int K, class T>
__global__ void __launch_bounds__(512) k_lu_forward_sub(LuDev F, const LuTask* __restrict__ tasks,
                                                        const int2* __restrict__ lev, const int* __restrict__ lptr,
                                                        int nb) {
  const int s = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  for (int l = lptr[s]; l < lptr[s + 1]; ++l) {
    const int2 rg = lev[l];
    if (nb == 1) {
      fwd_tasks<K, T>(F, tasks, rg.x + wave, rg.y, kSubWaves, lane);
    } else {
      for (int ti = rg.x + wave; ti < rg.y; ti += kSubWaves) {
        const LuTask t = tasks[ti];
        fwd_task_mr<T>(F, t, lane, nb);
      }
    }
    __syncthreads();  // this height's stores and atomics visible to the workgroup
  }
}
template <int K, class T, class TO>
__global__ void __launch_bounds__(512) k_lu_backward_sub(LuDev F, const LuTask* __restrict__ tasks,
                                                         const int2* __restrict__ lev, const int* __restrict__ lptr,
                                                         int nb, TO* __restrict__ out, long long ostride) {
  const int s = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  for (int l = lptr[s]; l < lptr[s + 1]; ++l) {
    const int2 rg = lev[l];
    if (nb == 1) {
      bwd_tasks<K, T, TO>(F, tasks, rg.x + wave, rg.y, kSubWaves, lane, out);
    } else {
      for (int ti = rg.x + wave; ti < rg.y; ti += kSubWaves) {
        const LuTask t = tasks[ti];
        bwd_task_mr<T, TO>(F, t, lane, nb, out, ostride);
      }
    }
    __syncthreads();  // this height's stores and atomics visible to the workgroup
  }
}

template <class T>
__global__ void k_zero(T* p, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = T(0);
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// per-batch max |v|: per-block maxima into partial[b * gridDim.x + block], then
// k_max_finish writes the bit pattern of the non-negative double to out[b]
__global__ void k_maxabs(const double* __restrict__ v, long long count, double* __restrict__ partial) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  v += (long long)blockIdx.y * count;
  double m = 0.0;
  for (; i < count; i += stride) m = nan_max(m, fabs(v[i]));
  m = block_max(m);
  if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = m;
}
__global__ void k_max_finish(const double* __restrict__ partial, int g, unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < g; i += blockDim.x) m = nan_max(m, partial[(long long)blockIdx.x * g + i]);
  m = block_max(m);
  if (threadIdx.x == 0) out[blockIdx.x] = (unsigned long long)__double_as_longlong(m);
}
// *out = sum of partial[i * nv + j] over i < g
__global__ void k_sum_finish_one(const double* __restrict__ partial, int g, int nv, int j, double* __restrict__ out) {
  double t = 0.0;
  for (int i = threadIdx.x; i < g; i += blockDim.x) t += partial[(long long)i * nv + j];
  t = block_sum(t);
  if (threadIdx.x == 0) *out = t;
}
// out[j] = sum of partial[i * nv + j] over i < g (one block per j)
__global__ void k_sum_finish(const double* __restrict__ partial, int g, int nv, double* __restrict__ out) {
  double t = 0.0;
  for (int i = threadIdx.x; i < g; i += blockDim.x) t += partial[(long long)i * nv + blockIdx.x];
  t = block_sum(t);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__device__ __forceinline__ double norm_value(const unsigned long long* norm, int b) {
  return norm ? __longlong_as_double((long long)norm[b]) : 1.0;
}

template <class T>
__global__ void k_add_unknowns(StencilLevel L, const T* __restrict__ e, const unsigned long long* __restrict__ norm,
                               double* __restrict__ phi) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n3 = (long long)L.n * L.n * L.n;
  if (c >= n3 || L.type[c] == 0) return;
  const int b = blockIdx.y;
  const double sc = norm_value(norm, b);
  phi[b * n3 + c] += sc * (double)e[b * n3 + c];
}

template <class T>
__global__ void k_scale_residual(long long n3, const double* __restrict__ s, const unsigned long long* __restrict__ norm,
                                 T* __restrict__ d) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n3) return;
  const int b = blockIdx.y;
  const double nv = norm_value(norm, b);
  const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
  d[b * n3 + c] = T(s[b * n3 + c] * inv);
}

__global__ void k_mask_unknowns(StencilLevel L, double* __restrict__ a) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n3 = (long long)L.n * L.n * L.n;
  if (c < n3 && L.type[c] == 0) a[blockIdx.y * n3 + c] = 0.0;
}

template <class T>
__global__ void k_copy_pairs(int count, const int2* __restrict__ pairs, T* __restrict__ a, long long stride) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  a += blockIdx.y * stride;
  if (t < count) a[pairs[t].x] = a[pairs[t].y];
}

__global__ void k_set_values(int count, const int* __restrict__ cells, const double* __restrict__ vals,
                             double* __restrict__ a) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) a[cells[t]] = vals[t];
}

// Learned-guess features on a coarse level of m^3 cells: x[V][0] = mean of r
// over the V's (n0/m)^3 fine cells times inv_norm, x[V][1] = volume fraction.
// Training pairs of the learned guess on an m^3 level of an n0^3 problem, for
// nb right-hand sides (r, phi: nb arrays of n0^3) with max|r_b| in norm[b] (bit
// patterns): x[b][V] = (mean of r_b over V's fine cells / max|r_b|, volume
// fraction), t[b][V] = phi_scale * (mean of phi_b over V's fine cells that
// carry an unknown) / max|r_b|, mask[b][V] = 1 where V holds such a cell.
__global__ void k_net_pairs(int n0, int m, const double* __restrict__ r, const double* __restrict__ phi,
                            const uint8_t* __restrict__ type0, const unsigned long long* __restrict__ norm,
                            const float* __restrict__ volfrac, double phi_scale, float* __restrict__ x,
                            float* __restrict__ t, uint8_t* __restrict__ mask) {
  const long long m3 = (long long)m * m * m, n3 = (long long)n0 * n0 * n0;
  const long long V = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (V >= m3) return;
  r += b * n3;
  phi += b * n3;
  const int f = n0 / m;
  const int I = (int)(V % m), J = (int)((V / m) % m), K = (int)(V / ((long long)m * m));
  double sr = 0.0, sp = 0.0;
  int cnt = 0;
  for (int dz = 0; dz < f; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const long long c = (I * f + dx) + (long long)n0 * ((J * f + dy) + (long long)n0 * (K * f + dz));
        sr += r[c];
        if (type0[c] != 0) {
          sp += phi[c];
          ++cnt;
        }
      }
  const double rn = __longlong_as_double((long long)norm[b]);
  const double inv = rn > 0.0 ? 1.0 / rn : 0.0;
  const long long o = b * m3 + V;
  x[2 * o] = (float)(sr / ((double)f * f * f) * inv);
  x[2 * o + 1] = volfrac[V];
  t[o] = cnt > 0 ? (float)(phi_scale * (sp / cnt) * inv) : 0.f;
  mask[o] = cnt > 0 ? 1 : 0;
}

__global__ void k_net_features(int n0, int m, const double* __restrict__ r, double inv_norm,
                               const float* __restrict__ volfrac, float* __restrict__ x) {
  long long V = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m3 = (long long)m * m * m;
  if (V >= m3) return;
  const int f = n0 / m;
  const int I = (int)(V % m), J = (int)((V / m) % m), K = (int)(V / ((long long)m * m));
  double s = 0.0;
  for (int dz = 0; dz < f; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx)
        s += r[(I * f + dx) + (long long)n0 * ((J * f + dy) + (long long)n0 * (K * f + dz))];
  x[2 * V] = (float)(s / ((double)f * f * f) * inv_norm);
  x[2 * V + 1] = volfrac[V];
}

// phi (level 0, unknown cells) = scale * trilinear interpolation of the
// cell-centred coarse field y (m^3) at the fine cell centres (clamped at the
// outer cells); 0 on cells without an unknown.
__global__ void k_prolong_trilinear(StencilLevel L0, int m, const float* __restrict__ y, double scale,
                                    double* __restrict__ phi) {
  const int n = L0.n;
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n3 = (long long)n * n * n;
  if (c >= n3) return;
  if (L0.type[c] == 0) {
    phi[c] = 0.0;
    return;
  }
  const int ii[3] = {(int)(c % n), (int)((c / n) % n), (int)(c / ((long long)n * n))};
  int lo[3], hi[3];
  double w[3];
  for (int a = 0; a < 3; ++a) {
    double X = (ii[a] + 0.5) * m / (double)n - 0.5;
    X = fmin(fmax(X, 0.0), (double)(m - 1));
    lo[a] = (int)floor(X);
    hi[a] = min(lo[a] + 1, m - 1);
    w[a] = X - lo[a];
  }
  double v = 0.0;
  for (int d = 0; d < 8; ++d) {
    const int ix = (d & 1) ? hi[0] : lo[0], iy = (d & 2) ? hi[1] : lo[1], iz = (d & 4) ? hi[2] : lo[2];
    const double wt = ((d & 1) ? w[0] : 1.0 - w[0]) * ((d & 2) ? w[1] : 1.0 - w[1]) * ((d & 4) ? w[2] : 1.0 - w[2]);
    v += wt * (double)y[ix + (long long)m * (iy + (long long)m * iz)];
  }
  phi[c] = scale * v;
}

// x = scale y on the cells of level Lm that carry an unknown, 0 elsewhere (a
// network output on that level's grid as the level's iterate)
__global__ void k_net_to_level(StencilLevel Lm, const float* __restrict__ y, double scale, double* __restrict__ x) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long m3 = (long long)Lm.n * Lm.n * Lm.n;
  if (c >= m3) return;
  x[c] = Lm.type[c] != 0 ? scale * (double)y[c] : 0.0;
}

// per-block partial sums of (w, V_i), i < NV, and (w, w) into
// partial[block * (NV + 1) + i]: w is read once for all the vectors
template <int NV>
__global__ void k_dots_multi(long long n3, const double* __restrict__ w, const double* __restrict__ V,
                             long long stride, double* __restrict__ partial) {
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n3;
       c += (long long)gridDim.x * blockDim.x) {
    const double wc = w[c];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += wc * V[i * stride + c];
    acc[NV] += wc * wc;
  }
#pragma unroll
  for (int i = 0; i <= NV; ++i) {
    const double t = block_sum(acc[i]);
    if (threadIdx.x == 0) partial[(long long)blockIdx.x * (NV + 1) + i] = t;
  }
}

// out = mode 0: sum_i coef[i] V_i;  1: out + sum;  2: out - sum;  3: scale: coef[0] * V_0
// and, if pmax / psq are given, per-block max |out| and sum out^2.  The nv <=
// kComboMax coefficients are staged in LDS; the vectors are read 8 at a time
// with all 8 loads (and out's) in flight.
constexpr int kComboMax = 128;
__global__ void __launch_bounds__(256) k_combo(long long n3, const double* __restrict__ V, long long stride,
                                               int nv, const double* __restrict__ coef, double* __restrict__ out,
                                               int mode, double* __restrict__ pmax, double* __restrict__ psq) {
  __shared__ double cs[kComboMax];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  double m = 0.0, q = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n3;
       c += (long long)gridDim.x * blockDim.x) {
    const double prev = (mode == 1 || mode == 2) ? out[c] : 0.0;
    double s0 = 0.0, s1 = 0.0;
    int i = 0;
    for (; i + 8 <= nv; i += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = V[(i + u) * stride + c];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        s0 += cs[i + u] * v[u];
        s1 += cs[i + u + 1] * v[u + 1];
      }
    }
    for (; i < nv; ++i) s0 += cs[i] * V[i * stride + c];
    const double sum = s0 + s1;
    const double o = mode == 1 ? prev + sum : (mode == 2 ? prev - sum : sum);
    if (out) out[c] = o;
    m = nan_max(m, fabs(o));
    q += o * o;
  }
  if (pmax) {
    m = block_max(m);
    if (threadIdx.x == 0) pmax[blockIdx.x] = m;
  }
  if (psq) {
    q = block_sum(q);
    if (threadIdx.x == 0) psq[blockIdx.x] = q;
  }
}

// plain copy (used to calibrate memory-traffic counters against a known size)
__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) dst[i] = src[i];
}

struct GaussQ {
  int q;
  double x[16], w[16];
};

__global__ void k_cell_average(int n, double h, double ox, double oy, double oz, FieldDesc f, int mode,
                               GaussQ G, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y * blockDim.y + threadIdx.y;
  int k = blockIdx.z;
  if (i >= n || j >= n) return;
  double cx = ox + (i + 0.5) * h, cy = oy + (j + 0.5) * h, cz = oz + (k + 0.5) * h;
  double acc = 0.0;
  for (int a = 0; a < G.q; ++a) {
    double z = cz + 0.5 * h * G.x[a];
    double sy = 0.0;
    for (int b = 0; b < G.q; ++b) {
      double y = cy + 0.5 * h * G.x[b];
      double sx = 0.0;
      for (int c = 0; c < G.q; ++c) sx += G.w[c] * field_value(f, cx + 0.5 * h * G.x[c], y, z, mode);
      sy += G.w[b] * sx;
    }
    acc += G.w[a] * sy;
  }
  out[i + (long)n * (j + (long)n * k)] = 0.125 * acc;
}

// Cut-cell integrals of several fields from line-piece rules: the workgroup of
// (cell c, field group y) walks the (piece, Gauss point) pairs of cell c, each
// thread evaluating every field of its group at its nodes.
constexpr int kPieceFields = 8;
constexpr int kPieceThreads = 256;

__global__ __launch_bounds__(kPieceThreads) void k_piece_integrals(const int* __restrict__ off,
                                                                   const PieceRec* __restrict__ pc, GaussQ G,
                                                                   const FieldDesc* __restrict__ fds, int nf,
                                                                   int mode, double* __restrict__ out) {
  const int c = blockIdx.x;
  const int f0 = blockIdx.y * kPieceFields;
  const int nfb = min(kPieceFields, nf - f0);
  const int p0 = off[c];
  const int total = (off[c + 1] - p0) * G.q;
  double acc[kPieceFields];
#pragma unroll
  for (int f = 0; f < kPieceFields; ++f) acc[f] = 0.0;
  for (int t = threadIdx.x; t < total; t += kPieceThreads) {
    const PieceRec P = pc[p0 + t / G.q];
    const int g = t % G.q;
    const double mid = 0.5 * (P.a + P.b), half = 0.5 * (P.b - P.a);
    const double wt = P.w * half * G.w[g];
    double x[3];
    int m = 0;
    for (int i = 0; i < 3; ++i) x[i] = (i == P.k) ? mid + half * G.x[g] : P.xo[m++];
#pragma unroll
    for (int f = 0; f < kPieceFields; ++f)
      if (f < nfb) acc[f] += wt * field_value(fds[f0 + f], x[0], x[1], x[2], mode);
  }
  __shared__ double part[kPieceFields][kPieceThreads / kWave];
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int f = 0; f < kPieceFields; ++f) {
    const double v = wave_sum(acc[f]);
    if ((threadIdx.x & (kWave - 1)) == 0) part[f][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < nfb) {
    double s = 0.0;
    for (int i = 0; i < kPieceThreads / kWave; ++i) s += part[threadIdx.x][i];
    out[(long long)c * nf + f0 + threadIdx.x] = s;
  }
}

inline dim3 grid3(int n) { return dim3((n + 63) / 64, (n + 3) / 4, n); }
inline dim3 grid_tiles(int n, int nb = 1) { return dim3(((n + 63) / 64) * ((n + 3) / 4) * n, nb); }
const dim3 kBlock3(64, 4, 1);
inline int blocks(long long count, int bs) { return (int)((count + bs - 1) / bs); }
// The regular-row kernels march in z from this grid size on (below, too few tiles to fill the
// chip); planes per workgroup: enough workgroups for the chip, at most 32
constexpr int kSmoMarchMin = 96;
inline int smo_march_planes(int n) {
  const long long tiles = (long long)((n + 63) / 64) * ((n + 3) / 4);
  const long long want = 8192;   // workgroups
  int kz = (int)std::min<long long>(32, std::max<long long>(8, (long long)n * tiles / want));
  return kz;
}
}  // namespace

void default_stencil_schedule(int n, int& march, int& kz) {
  march = n >= kSmoMarchMin ? 1 : 0;
  kz = smo_march_planes(n);
}

namespace {
inline dim3 march_grid(int n, int kz, int nb) {
  return dim3(((n + 63) / 64) * ((n + 3) / 4) * ((n + kz - 1) / kz), nb);
}
inline long long cube(int n) { return (long long)n * n * n; }
constexpr int kRedBlocks = 2048;   // blocks of the reductions (partial sums per block)

}  // namespace

template <class T>
void launch_smo1(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, int nb, hipStream_t st) {
  const int n = L.n;
  if (!L.march) {
    hipLaunchKernelGGL(k_smo1<T>, grid_tiles(n, nb), kBlock3, 0, st, L, T(omega), s, e_in, e_out);
    return;
  }
  const int kz = L.kz;
  hipLaunchKernelGGL(k_smo1_z<T>, march_grid(n, kz, nb), kBlock3, 0, st, L, T(omega), s, e_in, e_out, kz);
}
template <class T>
void launch_smo1_far(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, int nb,
                     hipStream_t st) {
  const int n = L.n;
  if (!L.march) {
    hipLaunchKernelGGL((k_smo1<T, true>), grid_tiles(n, nb), kBlock3, 0, st, L, T(omega), s, e_in, e_out);
    return;
  }
  const int kz = L.kz;
  hipLaunchKernelGGL(k_smo1_far_z<T>, march_grid(n, kz, nb), kBlock3, 0, st, L, T(omega), s, e_in, e_out, kz);
}
template <class T>
void launch_smo1_near(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, const int* cells,
                      int count, int nb, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_smo1_list<T>, dim3(blocks(count, 256), nb), dim3(256), 0, st, L, T(omega), s, e_in, e_out,
                     cells, count);
}
template <class T>
void launch_smo1_first(const StencilLevel& L, double omega, const T* s, T* e_out, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_smo1_first<T>, grid_tiles(L.n, nb), kBlock3, 0, st, L, T(omega), s, e_out);
}
void launch_stencil_residual(const StencilLevel& L, const double* r, const double* x, double* s, int nb,
                             hipStream_t st) {
  if (!L.march) {
    hipLaunchKernelGGL(k_stencil_residual, grid_tiles(L.n, nb), kBlock3, 0, st, L, r, x, s, 0);
    return;
  }
  const int kz = L.kz;
  hipLaunchKernelGGL(k_stencil_residual_z, march_grid(L.n, kz, nb), kBlock3, 0, st, L, r, x, s, kz);
}
void launch_stencil_apply(const StencilLevel& L, const double* x, double* y, hipStream_t st) {
  if (!L.march) {
    hipLaunchKernelGGL(k_stencil_residual, grid_tiles(L.n), kBlock3, 0, st, L, (const double*)nullptr, x, y, 1);
    return;
  }
  const int kz = L.kz;
  hipLaunchKernelGGL(k_stencil_apply_z, march_grid(L.n, kz, 1), kBlock3, 0, st, L, x, y, kz);
}
void launch_plg_residual(const PlgRows& P, const double* r, const double* x, double* s, int apply_only, int nb,
                         long long stride, hipStream_t st) {
  if (P.N2 == 0) return;
  hipLaunchKernelGGL(k_plg_residual, dim3(blocks((long long)P.N2 * kPlgLanes, 256), nb), dim3(256), 0, st, P, r, x,
                     s, apply_only, stride);
}
template <class T>
void launch_restrict(const StencilLevel& F, const StencilLevel& C, const T* s, const T* e, T* sc, int nb,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_restrict<T>, grid_tiles(C.n, nb), kBlock3, 0, st, F, C, s, e, sc);
}
void launch_fmg_restrict(const StencilLevel& F, const StencilLevel& C, const double* s, double* sc, int nb,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_fmg_restrict, grid_tiles(C.n, nb), kBlock3, 0, st, F, C, s, sc);
}
void launch_fmg_prolong(const StencilLevel& F, const StencilLevel& C, const double* xc, double* xf, int nb,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_fmg_prolong, grid_tiles(F.n, nb), kBlock3, 0, st, F, C, xc, xf);
}
template <class T>
void launch_prolong_add(const StencilLevel& F, int nc, const T* ec, T* ef, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_add<T>, grid_tiles(F.n, nb), kBlock3, 0, st, F, nc, ec, ef);
}
template <class T>
void launch_plg_b2(const PlgRows& P, const T* s, const T* e, T* y, long long stride, int nb, hipStream_t st) {
  if (P.N2 == 0) return;
  hipLaunchKernelGGL(k_plg_b2<T>, dim3(blocks((long long)P.N2 * kPlgLanes, 256), nb), dim3(256), 0, st, P, s, e, y,
                     stride);
}
template <class TS, class TY>
void launch_gather(int n, const int* row_cell, const TS* src, long long src_stride, TY* y, int nb, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_gather<TS, TY>), dim3(blocks(n, 256), nb), dim3(256), 0, st, n, row_cell, src, src_stride,
                     y);
}
inline dim3 wave_grid(int ntasks) { return dim3(blocks((long long)ntasks * kWave, 256)); }
// single right-hand side: at most wcap wavefronts, each looping over tasks
inline dim3 lu_grid(const LuTasks& S, int nb) {
  const int n = nb == 1 ? S.nF : S.nFm;
  return wave_grid(nb == 1 ? std::min(n, std::max(S.wcap, 4)) : n);
}
inline dim3 lu_grid_b(const LuTasks& S, int nb) {
  const int n = nb == 1 ? S.nB : S.nBm;
  return wave_grid(nb == 1 ? std::min(n, std::max(S.wcap, 4)) : n);
}

template <class T>
void launch_lu_forward(const LuDev& F, const LuTasks& S, int nb, hipStream_t st) {
  const int n = nb == 1 ? S.nF : S.nFm;
  if (n == 0) return;
  const LuTask* tk = nb == 1 ? S.ftask : S.ftask_m;
  const int kc = nb == 1 ? S.kc : 4;
  if (kc <= 4)
    hipLaunchKernelGGL((k_lu_forward<4, T>), lu_grid(S, nb), dim3(256), 0, st, F, tk, n, nb);
  else
    hipLaunchKernelGGL((k_lu_forward<8, T>), lu_grid(S, nb), dim3(256), 0, st, F, tk, n, nb);
}
template <class T, class TO>
void launch_lu_backward(const LuDev& F, const LuTasks& S, TO* out, long long out_stride, int nb, hipStream_t st) {
  const int n = nb == 1 ? S.nB : S.nBm;
  if (n == 0) return;
  const LuTask* tk = nb == 1 ? S.btask : S.btask_m;
  const int kc = nb == 1 ? S.kc : 4;
  if (kc <= 4)
    hipLaunchKernelGGL((k_lu_backward<4, T, TO>), lu_grid_b(S, nb), dim3(256), 0, st, F, tk, n, nb, out,
                       out_stride);
  else
    hipLaunchKernelGGL((k_lu_backward<8, T, TO>), lu_grid_b(S, nb), dim3(256), 0, st, F, tk, n, nb, out,
                       out_stride);
}
template <class T>
void launch_lu_forward_sub(const LuDev& F, const LuSub& S, int nb, hipStream_t st) {
  if (S.nsub == 0) return;
  const LuSubList& L = nb == 1 ? S.single : S.multi;
  const int kc = nb == 1 ? S.kc : 4;
  const dim3 grid(S.nsub), block(64 * kSubWaves);
  if (kc <= 4)
    hipLaunchKernelGGL((k_lu_forward_sub<4, T>), grid, block, 0, st, F, L.ftask, L.flev, L.fptr, nb);
  else
    hipLaunchKernelGGL((k_lu_forward_sub<8, T>), grid, block, 0, st, F, L.ftask, L.flev, L.fptr, nb);
}
template <class T, class TO>
void launch_lu_backward_sub(const LuDev& F, const LuSub& S, TO* out, long long out_stride, int nb, hipStream_t st) {
  if (S.nsub == 0) return;
  const LuSubList& L = nb == 1 ? S.single : S.multi;
  const int kc = nb == 1 ? S.kc : 4;
  const dim3 grid(S.nsub), block(64 * kSubWaves);
  if (kc <= 4)
    hipLaunchKernelGGL((k_lu_backward_sub<4, T, TO>), grid, block, 0, st, F, L.btask, L.blev, L.bptr, nb, out,
                       out_stride);
  else
    hipLaunchKernelGGL((k_lu_backward_sub<8, T, TO>), grid, block, 0, st, F, L.btask, L.blev, L.bptr, nb, out,
                       out_stride);
}
template <class T>
void launch_zero(T* p, long long count, hipStream_t st) {
  if (count == 0) return;
  int nb = (int)std::min<long long>(blocks(count, 256), 8192);
  hipLaunchKernelGGL(k_zero<T>, dim3(nb), dim3(256), 0, st, p, count);
}
// Workgroups of the one-launch sweeps: enough wavefronts to fill the chip
// (each loops over tickets); at most one per task.
constexpr int kFlowBlocks = 2048;
template <class T, class TO>
void launch_lu_flow(const LuDev& F, const LuFlow& W, TO* out, hipStream_t st) {
  launch_zero<int>(W.counters, W.ncounters, st);
  const int cap = W.max_waves > 0 ? std::max(1, W.max_waves / (256 / kWave)) : kFlowBlocks;
  const int gf = std::max(1, std::min(cap, blocks(W.fwd.ntask, 256 / kWave)));
  const int gb = std::max(1, std::min(cap, blocks(W.bwd.ntask, 256 / kWave)));
  if (W.fwd.ntask > 0) {
    if (W.kc <= 4)
      hipLaunchKernelGGL((k_lu_forward_flow<4, T>), dim3(gf), dim3(256), 0, st, F, W.ftask, W.fwd, W.limit);
    else
      hipLaunchKernelGGL((k_lu_forward_flow<8, T>), dim3(gf), dim3(256), 0, st, F, W.ftask, W.fwd, W.limit);
  }
  if (W.bwd.ntask > 0) {
    if (W.kc <= 4)
      hipLaunchKernelGGL((k_lu_backward_flow<4, T, TO>), dim3(gb), dim3(256), 0, st, F, W.btask, W.bwd, W.limit,
                         out);
    else
      hipLaunchKernelGGL((k_lu_backward_flow<8, T, TO>), dim3(gb), dim3(256), 0, st, F, W.btask, W.bwd, W.limit,
                         out);
  }
}
void launch_zero_u64(unsigned long long* p, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(blocks(count, 64)), dim3(64), 0, st, p, count);
}
void launch_maxabs(const double* v, long long count, int nb, unsigned long long* out, double* partial,
                   hipStream_t st) {
  const int g = (int)std::min<long long>(blocks(count, 256), kRedBlocks);
  hipLaunchKernelGGL(k_maxabs, dim3(g, nb), dim3(256), 0, st, v, count, partial);
  hipLaunchKernelGGL(k_max_finish, dim3(nb), dim3(256), 0, st, partial, g, out);
}
template <class T>
void launch_add_unknowns(const StencilLevel& L, const T* e, const unsigned long long* norm, double* phi, int nb,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_add_unknowns<T>, dim3(blocks(cube(L.n), 256), nb), dim3(256), 0, st, L, e, norm, phi);
}
template <class T>
void launch_scale_residual(long long n3, const double* s, const unsigned long long* norm, T* d, int nb,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_scale_residual<T>, dim3(blocks(n3, 256), nb), dim3(256), 0, st, n3, s, norm, d);
}
void launch_mask_unknowns(const StencilLevel& L, double* a, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_mask_unknowns, dim3(blocks(cube(L.n), 256), nb), dim3(256), 0, st, L, a);
}
template <class T>
void launch_copy_pairs(int count, const int2* pairs, T* a, long long stride, int nb, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_copy_pairs<T>, dim3(blocks(count, 256), nb), dim3(256), 0, st, count, pairs, a, stride);
}
template void launch_copy_pairs<double>(int, const int2*, double*, long long, int, hipStream_t);
template void launch_copy_pairs<float>(int, const int2*, float*, long long, int, hipStream_t);
__global__ void k_scatter_values(int count, const int* __restrict__ cells, const double* __restrict__ vals,
                                 double* __restrict__ a, long long stride, int nb, int add) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)count * nb) return;
  const int v = (int)(t / nb), b = (int)(t % nb);
  double* dst = a + b * stride + cells[v];
  *dst = add ? *dst + vals[t] : vals[t];
}
void launch_scatter_values(int count, const int* cells, const double* vals, double* a, long long stride, int nb,
                           int add, hipStream_t st) {
  if (count == 0 || nb == 0) return;
  hipLaunchKernelGGL(k_scatter_values, dim3(blocks((long long)count * nb, 256)), dim3(256), 0, st, count, cells, vals,
                     a, stride, nb, add);
}
void launch_set_values(int count, const int* cells, const double* vals, double* a, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_set_values, dim3(blocks(count, 256)), dim3(256), 0, st, count, cells, vals, a);
}
void launch_net_pairs(int n0, int m, int nb, const double* r, const double* phi, const uint8_t* type0,
                      const unsigned long long* norm, const float* volfrac, double phi_scale, float* x, float* t,
                      uint8_t* mask, hipStream_t st) {
  const long long m3 = (long long)m * m * m;
  hipLaunchKernelGGL(k_net_pairs, dim3(blocks(m3, 256), nb), dim3(256), 0, st, n0, m, r, phi, type0, norm, volfrac,
                     phi_scale, x, t, mask);
}
void launch_net_features(int n0, int m, const double* r, double inv_norm, const float* volfrac, float* x,
                         hipStream_t st) {
  const long long m3 = (long long)m * m * m;
  hipLaunchKernelGGL(k_net_features, dim3(blocks(m3, 256)), dim3(256), 0, st, n0, m, r, inv_norm, volfrac, x);
}
void launch_prolong_trilinear(const StencilLevel& L0, int m, const float* y, double scale, double* phi,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_trilinear, dim3(blocks(cube(L0.n), 256)), dim3(256), 0, st, L0, m, y, scale, phi);
}
void launch_net_to_level(const StencilLevel& Lm, const float* y, double scale, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_net_to_level, dim3(blocks(cube(Lm.n), 256)), dim3(256), 0, st, Lm, y, scale, x);
}
void launch_combo(long long n3, const double* V, long long stride, int nv, const double* coef, double* out, int mode,
                  unsigned long long* amax, double* sumsq, double* partial, hipStream_t st) {
  if (nv < 1 || nv > kComboMax) throw std::invalid_argument("launch_combo: vector count out of range");
  const int g = (int)std::min<long long>(blocks(n3, 256), kRedBlocks);
  double* pmax = amax ? partial : nullptr;
  double* psq = sumsq ? partial + kRedBlocks : nullptr;
  hipLaunchKernelGGL(k_combo, dim3(g), dim3(256), 0, st, n3, V, stride, nv, coef, out, mode, pmax, psq);
  if (amax) hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(256), 0, st, pmax, g, amax);
  if (sumsq) hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(256), 0, st, psq, g, 1, sumsq);
}
void launch_dots_norm(long long n3, const double* w, const double* V, long long stride, int nv, double* out,
                      double* partial, hipStream_t st) {
  const int g = (int)std::min<long long>(blocks(n3, 256), kRedBlocks);
  if (nv == 0) {
    hipLaunchKernelGGL(k_dots_multi<0>, dim3(g), dim3(256), 0, st, n3, w, V, stride, partial);
    hipLaunchKernelGGL(k_sum_finish_one, dim3(1), dim3(256), 0, st, partial, g, 1, 0, out);
    return;
  }
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int k = std::min(8, nv - i0);
    const double* Vi = V + (long long)i0 * stride;
    switch (k) {
#define CC_DOTS_CASE(K)                                                                   \
  case K:                                                                                 \
    hipLaunchKernelGGL(k_dots_multi<K>, dim3(g), dim3(256), 0, st, n3, w, Vi, stride, partial); \
    break;
      CC_DOTS_CASE(0) CC_DOTS_CASE(1) CC_DOTS_CASE(2) CC_DOTS_CASE(3) CC_DOTS_CASE(4) CC_DOTS_CASE(5)
      CC_DOTS_CASE(6) CC_DOTS_CASE(7) CC_DOTS_CASE(8)
#undef CC_DOTS_CASE
    }
    // out[i0 .. i0 + k - 1] are the projections; the chunk's norm slot is
    // written only by the last chunk, at out[nv]
    const int last = i0 + k >= nv;
    hipLaunchKernelGGL(k_sum_finish, dim3(k), dim3(256), 0, st, partial, g, k + 1, out + i0);
    if (last) hipLaunchKernelGGL(k_sum_finish_one, dim3(1), dim3(256), 0, st, partial, g, k + 1, k, out + nv);
  }
}
void launch_copy(long long count, const double* src, double* dst, hipStream_t st) {
  if (count == 0) return;
  int g = (int)std::min<long long>(blocks(count, 256), 16384);
  hipLaunchKernelGGL(k_copy, dim3(g), dim3(256), 0, st, src, dst, count);
}
void launch_piece_integrals(int ncell, const int* off, const PieceRec* pieces, int q, const FieldDesc* fds, int nf,
                            int mode, double* out, hipStream_t st) {
  if (ncell == 0 || nf == 0) return;
  if (q > 16) throw std::runtime_error("launch_piece_integrals: at most 16 Gauss points");
  GaussQ G;
  G.q = q;
  std::vector<double> x, w;
  gauss_legendre(q, x, w);
  for (int i = 0; i < q; ++i) {
    G.x[i] = x[i];
    G.w[i] = w[i];
  }
  hipLaunchKernelGGL(k_piece_integrals, dim3(ncell, (nf + kPieceFields - 1) / kPieceFields), dim3(kPieceThreads), 0,
                     st, off, pieces, G, fds, nf, mode, out);
}
void launch_cell_average(int n, double h, const double* origin, const FieldDesc& f, int mode, int q, double* out,
                         hipStream_t st) {
  GaussQ G;
  G.q = q;
  std::vector<double> x, w;
  gauss_legendre(q, x, w);
  for (int i = 0; i < q; ++i) {
    G.x[i] = x[i];
    G.w[i] = w[i];
  }
  hipLaunchKernelGGL(k_cell_average, grid3(n), kBlock3, 0, st, n, h, origin[0], origin[1], origin[2], f, mode, G,
                     out);
}

#define CC_INST(T)                                                                                            \
  template void launch_smo1<T>(const StencilLevel&, double, const T*, const T*, T*, int, hipStream_t);        \
  template void launch_smo1_first<T>(const StencilLevel&, double, const T*, T*, int, hipStream_t);           \
  template void launch_smo1_far<T>(const StencilLevel&, double, const T*, const T*, T*, int, hipStream_t);    \
  template void launch_smo1_near<T>(const StencilLevel&, double, const T*, const T*, T*, const int*, int, int, \
                                    hipStream_t);                                                             \
  template void launch_restrict<T>(const StencilLevel&, const StencilLevel&, const T*, const T*, T*, int,     \
                                   hipStream_t);                                                              \
  template void launch_prolong_add<T>(const StencilLevel&, int, const T*, T*, int, hipStream_t);              \
  template void launch_plg_b2<T>(const PlgRows&, const T*, const T*, T*, long long, int, hipStream_t);        \
  template void launch_zero<T>(T*, long long, hipStream_t);                                                   \
  template void launch_lu_forward<T>(const LuDev&, const LuTasks&, int, hipStream_t);                        \
  template void launch_lu_forward_sub<T>(const LuDev&, const LuSub&, int, hipStream_t);                      \
  template void launch_add_unknowns<T>(const StencilLevel&, const T*, const unsigned long long*, double*, int, \
                                       hipStream_t);                                                          \
  template void launch_scale_residual<T>(long long, const double*, const unsigned long long*, T*, int,        \
                                         hipStream_t);
CC_INST(double)
CC_INST(float)
#undef CC_INST
template void launch_lu_backward<double, double>(const LuDev&, const LuTasks&, double*, long long, int,
                                                 hipStream_t);
template void launch_zero<int>(int*, long long, hipStream_t);
template void launch_lu_flow<double, double>(const LuDev&, const LuFlow&, double*, hipStream_t);
template void launch_lu_flow<double, float>(const LuDev&, const LuFlow&, float*, hipStream_t);
template void launch_lu_flow<float, float>(const LuDev&, const LuFlow&, float*, hipStream_t);
template void launch_lu_backward<double, float>(const LuDev&, const LuTasks&, float*, long long, int, hipStream_t);
template void launch_lu_backward<float, float>(const LuDev&, const LuTasks&, float*, long long, int, hipStream_t);
template void launch_lu_backward_sub<double, double>(const LuDev&, const LuSub&, double*, long long, int, hipStream_t);
template void launch_lu_backward_sub<double, float>(const LuDev&, const LuSub&, float*, long long, int, hipStream_t);
template void launch_lu_backward_sub<float, float>(const LuDev&, const LuSub&, float*, long long, int, hipStream_t);
template void launch_gather<double, double>(int, const int*, const double*, long long, double*, int, hipStream_t);
template void launch_gather<float, double>(int, const int*, const float*, long long, double*, int, hipStream_t);

// ------------------------------------------------ FV-PLG least-squares fits
// The weighted fit of an FV-PLG row (Sec. 2.3, with the lattice of Sec. 4.1):
// the row is c = ell^T (W^1/2 A)^+ W^1/2, i.e. c_i = w_i^1/2 y_i with y the
// minimum-norm solution of (W^1/2 A)^T y = ell.  One wavefront per system:
// Householder QR of the m x 35 matrix B = W^1/2 A in LDS (column-major, the
// reflector of column k kept below its diagonal), R^T u = ell by forward
// substitution, then y = Q [u; 0] by the reflectors in reverse.
constexpr int kLsqCols = 35;
__global__ void __launch_bounds__(64) k_plg_lsq(int nsys, const int* __restrict__ off, const double* __restrict__ A,
                                                const double* __restrict__ ell, double* __restrict__ y,
                                                int* __restrict__ ok, int mmax) {
  extern __shared__ double lds[];
  const int s = blockIdx.x;
  if (s >= nsys) return;
  const int lane = threadIdx.x;
  const int r0 = off[s], m = off[s + 1] - r0;
  // column stride odd in doubles, so the lanes' columns fall in different banks
  const int ms = mmax | 1;
  double* a = lds;                                  // a[c * ms + r]
  double* yv = lds + (size_t)kLsqCols * ms;         // y (m)
  __shared__ double vd[kLsqCols], vv[kLsqCols], rd[kLsqCols], u[kLsqCols];
  const double* As = A + (size_t)r0 * kLsqCols;
  double amax = 0.0;
  for (int idx = lane; idx < m * kLsqCols; idx += kWave) {
    const double v = As[idx];
    a[(idx % kLsqCols) * ms + idx / kLsqCols] = v;
    amax = fmax(amax, fabs(v));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, kWave));
  __syncthreads();
  bool good = m >= kLsqCols;
  for (int k = 0; k < kLsqCols && good; ++k) {
    double* ak = a + (size_t)k * ms;
    double part = 0.0;
    for (int r = k + lane; r < m; r += kWave) part += ak[r] * ak[r];
    const double nrm2 = wave_sum(part);
    const double nrm = sqrt(nrm2);
    const double x0 = ak[k];
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vn = v0 * v0 + (nrm2 - x0 * x0);   // |x - alpha e_k|^2
    __syncthreads();
    if (lane == 0) {
      vd[k] = v0;
      vv[k] = vn;
      rd[k] = vn > 0.0 ? alpha : x0;
    }
    // columns c > k, one lane each: c <- c - (2 v.c / v.v) v
    const int c = lane;
    if (vn > 0.0 && c > k && c < kLsqCols) {
      double* ac = a + (size_t)c * ms;
      double dot = v0 * ac[k];
      for (int r = k + 1; r < m; ++r) dot += ak[r] * ac[r];
      const double f = 2.0 * dot / vn;
      ac[k] -= f * v0;
      for (int r = k + 1; r < m; ++r) ac[r] -= f * ak[r];
    }
    __syncthreads();
    if (!(fabs(rd[k]) > 1e-13 * amax)) good = false;
  }
  if (!good) {
    if (lane == 0) ok[s] = 0;
    return;
  }
  // R^T u = ell: R[i][k] = a[k][i] for i < k, R[k][k] = rd[k]
  for (int k = 0; k < kLsqCols; ++k) {
    double part = lane < k ? a[(size_t)k * ms + lane] * u[lane] : 0.0;
    const double sdot = wave_sum(part);
    if (lane == 0) u[k] = (ell[(size_t)s * kLsqCols + k] - sdot) / rd[k];
    __syncthreads();
  }
  for (int r = lane; r < m; r += kWave) yv[r] = r < kLsqCols ? u[r] : 0.0;
  __syncthreads();
  for (int k = kLsqCols - 1; k >= 0; --k) {
    if (!(vv[k] > 0.0)) continue;
    const double* ak = a + (size_t)k * ms;
    double part = 0.0;
    for (int r = k + 1 + lane; r < m; r += kWave) part += ak[r] * yv[r];
    const double dot = wave_sum(part) + vd[k] * yv[k];
    const double f = 2.0 * dot / vv[k];
    __syncthreads();
    for (int r = k + 1 + lane; r < m; r += kWave) yv[r] -= f * ak[r];
    if (lane == 0) yv[k] -= f * vd[k];
    __syncthreads();
  }
  for (int r = lane; r < m; r += kWave) y[r0 + r] = yv[r];
  if (lane == 0) ok[s] = 1;
}

void plg_lsq_device(int nsys, const int* off, const double* A, const double* ell, double* y, int* ok,
                    hipStream_t st) {
  if (nsys <= 0) return;
  int mmax = 0;
  for (int s = 0; s < nsys; ++s) mmax = std::max(mmax, off[s + 1] - off[s]);
  const size_t lds = ((size_t)kLsqCols * (mmax | 1) + mmax) * sizeof(double);
  if (lds > 60 * 1024) fail(CC_EPLG, "an FV-PLG fit with " + std::to_string(mmax) + " sites exceeds the device kernel's LDS");
  const long long rows = off[nsys];
  int* d_off = nullptr;
  int* d_ok = nullptr;
  double *d_A = nullptr, *d_ell = nullptr, *d_y = nullptr;
  auto chk = [](hipError_t e) {
    if (e != hipSuccess) fail(CC_EDEVICE, std::string("FV-PLG fits: ") + hipGetErrorString(e));
  };
  chk(hipMalloc(&d_off, (nsys + 1) * sizeof(int)));
  chk(hipMalloc(&d_ok, nsys * sizeof(int)));
  chk(hipMalloc(&d_A, rows * kLsqCols * sizeof(double)));
  chk(hipMalloc(&d_ell, (size_t)nsys * kLsqCols * sizeof(double)));
  chk(hipMalloc(&d_y, rows * sizeof(double)));
  chk(hipMemcpyAsync(d_off, off, (nsys + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  chk(hipMemcpyAsync(d_A, A, rows * kLsqCols * sizeof(double), hipMemcpyHostToDevice, st));
  chk(hipMemcpyAsync(d_ell, ell, (size_t)nsys * kLsqCols * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_plg_lsq, dim3(nsys), dim3(kWave), lds, st, nsys, d_off, d_A, d_ell, d_y, d_ok, mmax);
  chk(hipGetLastError());
  chk(hipMemcpyAsync(y, d_y, rows * sizeof(double), hipMemcpyDeviceToHost, st));
  chk(hipMemcpyAsync(ok, d_ok, nsys * sizeof(int), hipMemcpyDeviceToHost, st));
  chk(hipStreamSynchronize(st));
  (void)hipFree(d_off);
  (void)hipFree(d_ok);
  (void)hipFree(d_A);
  (void)hipFree(d_ell);
  (void)hipFree(d_y);
}

// The allocation-free entry points' scratch.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address that
// hipGetSymbolAddress returns for the current device may reach a kernel or a
// copy.  Each GPU holds its own copy of the array at its own address.
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void noalloc_scratch(int device, double** ptr, long long* capacity) {
  if (device < 0 || device >= kMaxDevices) fail(CC_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) fail(CC_EDEVICE, "scratch: the device is not current");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      fail(CC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  *capacity = kNoAllocScratchDoubles;
}

}  // namespace cc
